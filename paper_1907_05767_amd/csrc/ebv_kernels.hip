/*
 * HIP kernels and their launchers for libebv (gfx950).
 *
 * Dense single system (Eq. 6-a/6-c applied 64 steps at a time):
 *   k_step    one launch per 64-wide block step (the default schedule): the
 *             diagonal tile's update and factor, the panel tiles solved
 *             against it strip by strip, and the update of the trailing
 *             region's column classes that are due, as ticket-ordered work
 *             items;
 *   k_diag, k_panel, k_update: the schedule without look-ahead (one launch
 *             per phase), kept as a tuning choice.
 * Triangular solves (Eq. 1): k_trsv, three workgroups per 64-row block (two
 *   helpers that take two thirds of the older blocks' contributions, and the
 *   block's own); workgroups take tickets in solve order, invert their
 *   diagonal block while the earlier blocks are solved, and wait for the
 *   blocks they depend on through marked exchange rows and a solved-blocks
 *   counter (no grid barrier).
 * Batches: one workgroup per system (k_lu_batch, k_solve_batch, and the
 *   persistent k_batched for ragged sizes, which takes systems from a queue
 *   in the EbV largest-with-smallest order).
 * Band, adjoint and mixed-precision helpers follow.
 */
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "ebv_device.hpp"
#include "ebv_internal.hpp"

namespace ebv {

/* ------------------------------------------------------------ utility --- */

__global__ void k_fill_i32(int *p, int64_t count, int value)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

hipError_t fill_i32(int *p, int64_t count, int value, hipStream_t st)
{
    if (count <= 0)
        return hipSuccess;
    int grid = (int)std::min<int64_t>((count + 255) / 256, 1024);
    hipLaunchKernelGGL(k_fill_i32, dim3(grid), dim3(256), 0, st, p, count, value);
    return hipGetLastError();
}

__global__ void k_fill_u64(unsigned long long *p, int64_t count, unsigned long long value)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

hipError_t fill_u64(unsigned long long *p, int64_t count, unsigned long long value, hipStream_t st)
{
    if (count <= 0)
        return hipSuccess;
    int grid = (int)std::min<int64_t>((count + 255) / 256, 1024);
    hipLaunchKernelGGL(k_fill_u64, dim3(grid), dim3(256), 0, st, p, count, value);
    return hipGetLastError();
}

__global__ void k_fold_status(const int *status, int32_t *info)
{
    if (threadIdx.x == 0) {
        const int v = *status;
        if (v)
            *info = -v;
    }
}

hipError_t fold_status(const int *status, int32_t *info, hipStream_t st)
{
    if (!info)
        return hipSuccess;
    hipLaunchKernelGGL(k_fold_status, dim3(1), dim3(64), 0, st, status, info);
    return hipGetLastError();
}

/* Fill count elements of an exchange buffer with the unsolved mark (as raw
 * bits: the mark never passes through floating-point registers). */
template <typename T> static hipError_t fill_unsolved(T *p, int64_t count, hipStream_t st)
{
    if (count <= 0)
        return hipSuccess;
    if (sizeof(T) == 8) {
        const int grid = (int)std::min<int64_t>((count + 255) / 256, 1024);
        hipLaunchKernelGGL(k_fill_u64, dim3(grid), dim3(256), 0, st, reinterpret_cast<unsigned long long *>(p),
                           count, kUnsolvedMark64);
        return hipGetLastError();
    }
    return fill_i32(reinterpret_cast<int *>(p), count, (int)kUnsolvedMark32, st);
}

/* ------------------------------------------------------- dense factor --- */

/* LDS of the workgroup that factors a diagonal tile: the tile, the packed
 * inverses of its factors, the pivot reciprocals. */
template <typename T> struct DiagSmem {
    T S[TB * LDT];
    T P[TB * LDT];
    T rinv[TB];
    T aux[32 + 256];
    int zflag;
    int avail;
};

/*
 * Diagonal tile of a block step: factor the 64x64 tile at (d0, d0), already
 * staged in sm.S with identity padding (tile_lu16), store it in place, and
 * store the packed inverses of its factors (tile_inv16) to Pg (64 x 64,
 * pitch TB) for the panel solves of the next launch (for the last tile only
 * when inv_last: right-hand sides ride along).  Run by the single
 * workgroup of k_diag (the first step) and by the extra workgroup of
 * k_update (every later step).
 */
template <typename T>
__device__ __forceinline__ void diag_tile(T *__restrict__ A, int64_t lda, int n, int d0, int32_t *info,
                                          T *__restrict__ Pg, DiagSmem<T> &sm, bool inv_last)
{
    const int dw = min(TB, n - d0);
    T *Add = A + (int64_t)d0 * lda + d0;
    const int z = tile_lu16(sm.S, sm.rinv, sm.aux, dw, &sm.zflag);
    lds_store_tile(sm.S, Add, lda, dw, dw);
    if (threadIdx.x == 0 && info && z && *info == 0)
        *info = d0 + z;
    if (d0 + dw >= n && !inv_last)
        return; /* last tile: no panel follows */
    tile_inv16(sm.S, sm.rinv, sm.P);
    tile_xfer<T>([&](int r, int c) { return sm.P[r * LDT + c]; }, [&](int r, int c, T v) { Pg[r * TB + c] = v; });
}

template <typename T>
__global__ __launch_bounds__(NT) void k_diag(T *__restrict__ A, int64_t lda, int n, int d0, int32_t *info,
                                             T *__restrict__ Pg, int inv_last)
{
    __shared__ DiagSmem<T> sm;
    const int dw = min(TB, n - d0);
    stage_tile_identity(sm.S, A + (int64_t)d0 * lda + d0, lda, dw, dw);
    __syncthreads();
    diag_tile(A, lda, n, d0, info, Pg, sm, inv_last != 0);
}

/*
 * Panel solves of one block step, as products with the inverses of the
 * diagonal tile's factors (Pg, packed by tile_inv16): a U block right of the
 * diagonal tile, U_kj = L_kk^{-1} A_kj, or an L block below it,
 * L_ik = A_ik U_kk^{-1}; one 64x64 block per workgroup, on the matrix cores.
 * With right-hand sides B (nrhs columns) the last workgroups also take the
 * forward-substitution step of Eq. 1 for block row k, Y_k = L_kk^{-1} B_k,
 * 64 columns each: B is carried as extra columns of the elimination.
 */
template <typename T>
__global__ __launch_bounds__(NT) void k_panel(T *__restrict__ A, int64_t lda, int n, int k0,
                                              const T *__restrict__ Pg, T *__restrict__ B, int64_t ldb, int nrhs)
{
    __shared__ T sP[TB * LDT], sX[TB * LDT];
    const int kw = min(TB, n - k0);
    const int nrem = (n - k0 - kw + TB - 1) / TB;
    const int t = blockIdx.x;
    tile_xfer<T>([&](int r, int c) { return Pg[r * TB + c]; }, [&](int r, int c, T v) { sP[r * LDT + c] = v; });
    if (t < nrem) {
        const int j0 = k0 + kw + t * TB, jw = min(TB, n - j0);
        T *G = A + (int64_t)k0 * lda + j0;
        stage64<T, false>(sX, G, lda, kw, jw);
        __syncthreads();
        wg_gemm64f<T, true>(DenseC<T>{G, lda, kw, jw}, InvL<T>{sP},
                            [&](int k, int c) { return sX[k * LDT + c]; });
    } else if (t < 2 * nrem) {
        const int i0 = k0 + kw + (t - nrem) * TB, iw = min(TB, n - i0);
        T *G = A + (int64_t)i0 * lda + k0;
        stage64<T, false>(sX, G, lda, iw, kw);
        __syncthreads();
        wg_gemm64f<T, true>(DenseC<T>{G, lda, iw, kw}, [&](int r, int k) { return sX[r * LDT + k]; },
                            InvU<T>{sP});
    } else {
        const int c0 = (t - 2 * nrem) * TB, cw = min(TB, nrhs - c0);
        T *G = B + (int64_t)k0 * ldb + c0;
        stage64<T, false>(sX, G, ldb, kw, cw);
        __syncthreads();
        wg_gemm64f<T, true>(DenseC<T>{G, ldb, kw, cw}, InvL<T>{sP},
                            [&](int k, int c) { return sX[k * LDT + c]; });
    }
}

/*
 * Trailing update A22 -= L21 U12 of one BM x BN tile (rows r0.., columns
 * c0.., K = kw <= 64 columns of the panel at k0): the rank-kw update of
 * Eq. 6-c on the matrix cores.  The tile is held in registers for the whole
 * K loop (read once, written once); 4 waves, each a (BM/2) x (BN/2) block of
 * 16x16 matrix-core tiles.  K runs in BK-deep chunks through double-buffered
 * LDS: the next chunk's global loads are in flight while the current one
 * feeds the matrix cores.  L21 is kept row-major in LDS with an odd pitch
 * (conflict-free column reads), U12 row-major.  The top-left skip x skip
 * corner of the tile is not stored (it belongs to another workgroup).
 */
template <typename T, int BM, int BN, int BK> struct UpdateTile {
    static constexpr int PA = BK + 1, PB = BN + 4;
    static constexpr size_t LDS = sizeof(T) * 2 * (BM * PA + BK * PB);
};

template <typename T, int BM, int BN, int BK>
__device__ __forceinline__ void update_tile(T *__restrict__ A, int64_t lda, int n, int k0, int kw, int r0, int c0,
                                            int skip, char *lds_raw)
{
    typedef typename vec4<T>::type V;
    constexpr int WM = BM / 2, WN = BN / 2, MB = WM / 16, NB = WN / 16;
    constexpr int PA = UpdateTile<T, BM, BN, BK>::PA, PB = UpdateTile<T, BM, BN, BK>::PB;
    constexpr int EA = BM * BK / NT, EB = BK * BN / NT; /* elements per thread per chunk */
    static_assert(BK % EA == 0 && BN % EB == 0, "chunk split");
    T(*sA)[BM * PA] = reinterpret_cast<T(*)[BM * PA]>(lds_raw);
    T(*sB)[BK * PB] = reinterpret_cast<T(*)[BK * PB]>(lds_raw + sizeof(T) * 2 * BM * PA);
    const int nr = min(BM, n - r0), nc = min(BN, n - c0);

    const int t = threadIdx.x, w = wave_id(), l = t & 63, lr = l & 15, lk = l >> 4;
    const int wm = (w >> 1) * WM, wn = (w & 1) * WN;

    /* this thread's share of a chunk: A rows ar, k offset ak..ak+EA; B row bk, cols bc..bc+EB */
    const int ar = t / (BK / EA), ak = (t % (BK / EA)) * EA;
    const int bk = t / (BN / EB), bc = (t % (BN / EB)) * EB;
    T ra[EA], rb[EB];
    auto fetch = [&](int kc) {
#pragma unroll
        for (int e = 0; e < EA; ++e) {
            const int kk = kc + ak + e;
            ra[e] = (ar < nr && kk < kw) ? A[(int64_t)(r0 + ar) * lda + k0 + kk] : T(0);
        }
#pragma unroll
        for (int e = 0; e < EB; ++e) {
            const int kk = kc + bk;
            rb[e] = (bc + e < nc && kk < kw) ? A[(int64_t)(k0 + kk) * lda + c0 + bc + e] : T(0);
        }
    };
    auto park = [&](int buf) {
#pragma unroll
        for (int e = 0; e < EA; ++e)
            sA[buf][ar * PA + ak + e] = ra[e];
#pragma unroll
        for (int e = 0; e < EB; ++e)
            sB[buf][bk * PB + bc + e] = rb[e];
    };

    fetch(0);
    V acc[MB][NB];
#pragma unroll
    for (int bi = 0; bi < MB; ++bi)
#pragma unroll
        for (int bj = 0; bj < NB; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = wm + 16 * bi + acc_row<T>(lk, r), col = wn + 16 * bj + lr;
                acc[bi][bj][r] = (row < nr && col < nc) ? A[(int64_t)(r0 + row) * lda + c0 + col] : T(0);
            }
    park(0);
    __syncthreads();
    const int nchunks = (kw + BK - 1) / BK;
    for (int c = 0; c < nchunks; ++c) {
        const int buf = c & 1;
        if (c + 1 < nchunks)
            fetch((c + 1) * BK);
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            T av[MB], bv[NB];
#pragma unroll
            for (int bi = 0; bi < MB; ++bi)
                av[bi] = -sA[buf][(wm + 16 * bi + lr) * PA + kk + lk];
#pragma unroll
            for (int bj = 0; bj < NB; ++bj)
                bv[bj] = sB[buf][(kk + lk) * PB + wn + 16 * bj + lr];
#pragma unroll
            for (int bi = 0; bi < MB; ++bi)
#pragma unroll
                for (int bj = 0; bj < NB; ++bj)
                    acc[bi][bj] = mfma16(av[bi], bv[bj], acc[bi][bj]);
        }
        if (c + 1 < nchunks)
            park(buf ^ 1);
        __syncthreads();
    }
#pragma unroll
    for (int bi = 0; bi < MB; ++bi)
#pragma unroll
        for (int bj = 0; bj < NB; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = wm + 16 * bi + acc_row<T>(lk, r), col = wn + 16 * bj + lr;
                if (row < nr && col < nc && !(row < skip && col < skip))
                    A[(int64_t)(r0 + row) * lda + c0 + col] = acc[bi][bj][r];
            }
}

/* Tile index -> position: tiles are dealt to the 8 XCDs in contiguous runs
 * (workgroups are dispatched round-robin over XCDs), so neighbouring tiles
 * share an XCD's L2. */
__device__ __forceinline__ int xcd_tile(int b, int ntiles)
{
    const int xcd = b & 7, per = ntiles >> 3, rem = ntiles & 7;
    return xcd * per + min(xcd, rem) + (b >> 3);
}

/*
 * One block step of the launch-per-phase factor: the trailing update of the
 * region right of and below the panel at k0 in BM x BN tiles, plus one extra
 * workgroup that updates, factors and inverts the next diagonal tile (the
 * tile workgroup covering that corner does not store it), plus (with
 * right-hand sides) workgroups for B_i -= L_ik Y_k.
 */
template <typename T, int BM, int BN, int BK>
__global__ __launch_bounds__(NT, 2) void k_update(T *__restrict__ A, int64_t lda, int n, int k0, int kw,
                                                  int32_t *info, T *__restrict__ Pg, T *__restrict__ B,
                                                  int64_t ldb, int nrhs)
{
    constexpr size_t GEMM_LDS = UpdateTile<T, BM, BN, BK>::LDS;
    constexpr size_t LDS_BYTES = GEMM_LDS > sizeof(DiagSmem<T>) ? GEMM_LDS : sizeof(DiagSmem<T>);
    __shared__ __attribute__((aligned(16))) char lds_raw[LDS_BYTES];

    const int i0 = k0 + kw, m = n - i0;
    const int tiles_n = (m + BN - 1) / BN;
    const int ntiles = ((m + BM - 1) / BM) * tiles_n;
    const int b = blockIdx.x;
    const int dw = min(TB, m); /* next diagonal tile: rows/cols i0..i0+dw */
    if (b == ntiles) {
        /* the extra workgroup: update the next diagonal tile itself (in
         * registers, then LDS) and factor it in place (the next block step's
         * diagonal tile); the tile workgroup covering it does not store that
         * corner */
        DiagSmem<T> &sm = *reinterpret_cast<DiagSmem<T> *>(lds_raw);
        const DenseC<T> C{A + (int64_t)i0 * lda + i0, lda, dw, dw};
        Acc64<T> acc;
        acc64_load(acc, C);
        stage64<T, false>(sm.S, A + (int64_t)i0 * lda + k0, lda, dw, kw);
        stage64<T, false>(sm.P, A + (int64_t)k0 * lda + i0, lda, kw, dw);
        __syncthreads();
        acc64_mma<T, true>(acc, [&](int r, int k) { return sm.S[r * LDT + k]; },
                           [&](int k, int c) { return sm.P[k * LDT + c]; });
        __syncthreads();
        acc64_store(acc, LdsTile<T>{sm.S});
        __syncthreads();
        if (threadIdx.x < TB && threadIdx.x >= dw) /* identity padding of a partial last tile */
            sm.S[threadIdx.x * (LDT + 1)] = T(1);
        __syncthreads();
        diag_tile(A, lda, n, i0, info, Pg, sm, B != nullptr);
        return;
    }
    if (b > ntiles) {
        /* right-hand-side workgroups: B_i -= L_ik Y_k for one 64-row block
         * below the panel and one 64-column chunk of B */
        DiagSmem<T> &sm = *reinterpret_cast<DiagSmem<T> *>(lds_raw);
        const int nbc = (nrhs + TB - 1) / TB, q = b - ntiles - 1;
        const int r0 = i0 + (q / nbc) * TB, c0 = (q % nbc) * TB;
        const int nr = min(TB, n - r0), nc = min(TB, nrhs - c0);
        stage64<T, true>(sm.S, A + (int64_t)r0 * lda + k0, lda, nr, kw);
        stage64<T, false>(sm.P, B + (int64_t)k0 * ldb + c0, ldb, kw, nc);
        __syncthreads();
        wg_gemm64(DenseC<T>{B + (int64_t)r0 * ldb + c0, ldb, nr, nc}, sm.S, sm.P);
        return;
    }
    const int tile = xcd_tile(b, ntiles);
    const int r0 = i0 + (tile / tiles_n) * BM, c0 = i0 + (tile % tiles_n) * BN;
    update_tile<T, BM, BN, BK>(A, lda, n, k0, kw, r0, c0, (r0 == i0 && c0 == i0) ? dw : 0, lds_raw);
}

/*
 * One block step of the look-ahead factor: launch s factors diagonal tile s
 * (rows/columns d0 = 64 s ...) and forms panel s, while it brings the
 * region right of and below tile s up to date.  Block column J belongs to
 * class J mod G; the steps not yet applied to class c are the last pend(c)
 * steps before s (pend(c) = byte c of pendp), and each tile applies all of
 * its column's pending steps at once (K = 64 pend(c)).  The region's tiles
 * are updated for class upd only (upd >= 0) or for every class (upd < 0);
 * B rows below block row s receive step s - 1 in every launch.
 * Work items are taken in ticket order (word 0 of the step's control words
 * w = ctl + 3 + 2 s):
 *   ticket 0     the diagonal tile: its pending update, then the factor
 *                (tile_lu16); the pack the panel items solve against (the
 *                factored tile, its 16 x 16 diagonal blocks replaced by the
 *                inverses of their factors) is published 16 columns at a
 *                time: while wave 0 factors panel p + 1 the other waves
 *                invert panel p's diagonal block and store the strip, each
 *                wave adding one to w[1] once its stores have landed (3 per
 *                strip), checked a panel later so that the factorization
 *                never waits for the stores;
 *   then         the first wave of BM x 64 region tiles (first_wave of
 *                them): tiles right of and below the panel, in the updated
 *                classes, update only;
 *   then         the panel tiles of step s -- U_sj = L_ss^{-1} A_sj and
 *                L_is = A_is U_ss^{-1} -- and Y_s = L_ss^{-1} B_s: each
 *                applies its own pending update first, then runs the block
 *                substitution against the pack, step p as soon as strip p
 *                is out (w[1] >= 3 (p + 1));
 *   last         the other region tiles, and (with B) B_i -= L_{i,s-1}
 *                Y_{s-1} below block row s.
 * The panel tiles start as soon as the first wave of region tiles frees
 * slots, not behind all of them.  The item they wait for (ticket 0) is
 * running before any of them starts and waits for nothing, so the wait
 * always ends (it is also bounded, reporting into ctl[0]).  The pack and
 * the flag are exchanged with device-coherent operations (store_coherent /
 * load_coherent, wait_solved).
 */
template <typename T, int BM, int BN, int BK>
__global__ __launch_bounds__(NT, 2) void k_step(T *__restrict__ A, int64_t lda, int n, int s, int G, int upd,
                                                int pendp, int first_wave, int32_t *info, T *__restrict__ Pg,
                                                T *__restrict__ B, int64_t ldb, int nrhs, int *ctl, long wlim)
{
    static_assert(BN == TB, "one block column per update tile (one class)");
    constexpr size_t GEMM_LDS = UpdateTile<T, BM, BN, BK>::LDS;
    constexpr size_t LDS_BYTES = GEMM_LDS > sizeof(DiagSmem<T>) ? GEMM_LDS : sizeof(DiagSmem<T>);
    __shared__ __attribute__((aligned(16))) char lds_raw[LDS_BYTES];
    __shared__ int s_ticket, s_avail;
    DiagSmem<T> &sm = *reinterpret_cast<DiagSmem<T> *>(lds_raw);

    const int d0 = s * TB, dw = min(TB, n - d0);
    /* pending rank of block column J (a multiple of 64) */
    auto kw_of = [&](int J) { return TB * ((pendp >> (8 * (J % G))) & 255); };
    const int kwB = s > 0 ? TB : 0;                /* B rows: one step behind */
    const int e0 = d0 + dw, m2 = n - e0;            /* region past the diagonal tile */
    const int nr2 = (m2 + TB - 1) / TB;             /* its block columns (and rows) */
    const int J0 = s + 1;                           /* its first block column */
    const int jfirst = upd < 0 ? 0 : ((upd - J0 % G) % G + G) % G; /* first updated column, from J0 */
    const int jstep = upd < 0 ? 1 : G;
    const int ncu = upd == -2 || jfirst >= nr2 ? 0 : (nr2 - jfirst + jstep - 1) / jstep;
    const int nrt = (m2 + BM - 1) / BM;
    const int nt2 = nrt * ncu;
    const int nbc = B ? (nrhs + TB - 1) / TB : 0;
    const int nb2 = kwB > 0 ? nr2 * nbc : 0;
    const int npan = 2 * nr2 + nbc; /* panel tiles of step s */
    int *status = ctl, *wstep = ctl + kCtlHead + 2 * s, *flag = wstep + 1;

    if (threadIdx.x == 0) {
        s_ticket = atomicAdd(wstep, 1);
        s_avail = 0;
    }
    __syncthreads();
    int q = s_ticket;
    if (q >= 1 + nt2 + nb2 + npan) { /* counter not reset: refuse */
        if (threadIdx.x == 0)
            atomicOr(status, 2);
        return;
    }

    if (q == 0) { /* the diagonal tile */
        const int kw = kw_of(s), k0 = d0 - kw;
        if (kw > 0) {
            /* its update in registers, K in 64-wide chunks staged in S (L) and P (U) */
            const DenseC<T> C{A + (int64_t)d0 * lda + d0, lda, dw, dw};
            Acc64<T> acc;
            acc64_load(acc, C);
            for (int h = 0; h < kw; h += TB) {
                stage64x2<T>(sm.S, A + (int64_t)d0 * lda + k0 + h, lda, dw, TB, sm.P, A + (int64_t)(k0 + h) * lda + d0,
                             lda, TB, dw);
                __syncthreads();
                acc64_mma<T, true>(acc, [&](int r, int k) { return sm.S[r * LDT + k]; },
                                   [&](int k, int c) { return sm.P[k * LDT + c]; });
                __syncthreads();
            }
            acc64_store(acc, LdsTile<T>{sm.S});
            __syncthreads();
            if (threadIdx.x < TB && threadIdx.x >= dw) /* identity padding of a partial last tile */
                sm.S[threadIdx.x * (LDT + 1)] = T(1);
            __syncthreads();
        } else {
            stage_tile_identity(sm.S, A + (int64_t)d0 * lda + d0, lda, dw, dw);
            __syncthreads();
        }
        T *Add = A + (int64_t)d0 * lda + d0;
        const bool pub = nr2 > 0 || nbc > 0;
        /* what the panel items read, published 16 columns at a time: for
         * panel q of the factored tile, role 0 and 1 the inverses of its
         * diagonal block's factors (to Pg), role 2 the block itself (to A,
         * read by no other item) and its L part below and U part to the
         * right (to A, device-coherent) */
        /* stage 0 issues this wave's part of panel q, stage 1 waits for its
         * stores and counts it */
        auto publish_panel = [&](int q, int role, int stage) __attribute__((always_inline)) {
            const int l = threadIdx.x & 63, b0 = 16 * q;
            if (stage == 1) {
                /* this wave's part of panel q has landed: count it (3 per panel) */
                if (role <= 2) {
                    __builtin_amdgcn_s_waitcnt(0);
                    if (l == 0)
                        __hip_atomic_fetch_add(flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                return;
            }
            auto put = [&](int i, int c, T v) __attribute__((always_inline)) {
                store_coherent(Pg + (b0 + i) * TB + b0 + c, v);
            };
            if (role == 0) {
                diag_block_inv<T, false>(sm.S, sm.rinv, q, put);
            } else if (role == 1) {
                diag_block_inv<T, true>(sm.S, sm.rinv, q, put);
            } else if (role == 2) {
                for (int idx = l; idx < 256; idx += 64) {
                    const int r = b0 + (idx >> 4), c = b0 + (idx & 15);
                    if (r < dw && c < dw)
                        Add[(int64_t)r * lda + c] = sm.S[r * LDT + c];
                }
                for (int idx = l; idx < (48 - b0) * 16; idx += 64) {
                    const int a = b0 + 16 + (idx >> 4), b = b0 + (idx & 15);
                    if (a < dw && b < dw) {
                        store_coherent(Add + (int64_t)a * lda + b, sm.S[a * LDT + b]);
                        store_coherent(Add + (int64_t)b * lda + a, sm.S[b * LDT + a]);
                    }
                }
            }
        };
        /* panels 0..2 are published by waves 1..3 while wave 0 factors the
         * next panel; the last one after the factorization */
        const int z = tile_lu16(sm.S, sm.rinv, sm.aux, dw, &sm.zflag, [&](int q, int stage) __attribute__((always_inline)) {
            if (pub)
                publish_panel(q, wave_id() - 1, stage);
        });
        if (threadIdx.x == 0 && info && z && *info == 0)
            *info = d0 + z;
        if (pub) {
            if (wave_id() >= 1) /* panel 2's stores, issued while panel 3 was factored */
                publish_panel(2, wave_id() - 1, 1);
            publish_panel(3, wave_id(), 0);
            publish_panel(3, wave_id(), 1);
        } else {
            lds_store_tile(sm.S, Add, lda, dw, dw);
        }
        return;
    }
    q -= 1;
    /* panel tile p of step s: 0..nr2-1 U tiles, nr2..2nr2-1 L tiles, then the
     * right-hand-side chunks of block row s */
    int kind, r0, c0, nr, nc, kw;
    T *G_;
    int64_t ldg;
    auto panel_tile = [&](int p) {
        if (p < nr2) {
            kind = 0;
            r0 = d0, c0 = e0 + p * TB;
            nr = dw, nc = min(TB, n - c0);
            G_ = A + (int64_t)r0 * lda + c0, ldg = lda;
            kw = kw_of(J0 + p);
        } else if (p < 2 * nr2) {
            kind = 1;
            r0 = e0 + (p - nr2) * TB, c0 = d0;
            nr = min(TB, n - r0), nc = dw;
            G_ = A + (int64_t)r0 * lda + c0, ldg = lda;
            kw = kw_of(s);
        } else {
            kind = 2;
            r0 = d0, c0 = (p - 2 * nr2) * TB;
            nr = dw, nc = min(TB, nrhs - c0);
            G_ = B + (int64_t)r0 * ldb + c0, ldg = ldb;
            kw = kwB;
        }
    };
    /* after the diagonal tile: the first wave of region tiles (first_wave of
     * them), then the panel tiles, then the other region tiles and the B
     * rows: the panel tiles start as soon as the first region tiles finish
     * instead of after all of them */
    const int n1 = min(nt2, first_wave);
    if (q >= n1 && q < n1 + npan) {
        q -= n1;
        goto panel;
    }
    if (q >= n1)
        q -= npan;
    if (q < nt2) { /* trailing tile of an updated class, update only */
        const int tile = xcd_tile(q, nt2);
        const int jc = jfirst + jstep * (tile % ncu);
        const int r0 = e0 + (tile / ncu) * BM, c0 = e0 + jc * TB;
        const int kw = kw_of(J0 + jc);
        update_tile<T, BM, BN, BK>(A, lda, n, d0 - kw, kw, r0, c0, 0, lds_raw);
        return;
    }
    q -= nt2;
    { /* B_i -= L_{i,s-1} Y_{s-1} for a 64-row block below block row s */
        const int r0 = e0 + (q / nbc) * TB, c0 = (q % nbc) * TB;
        const int nr = min(TB, n - r0), nc = min(TB, nrhs - c0);
        const int k0 = d0 - kwB;
        const DenseC<T> C{B + (int64_t)r0 * ldb + c0, ldb, nr, nc};
        Acc64<T> acc;
        acc64_load(acc, C);
        for (int h = 0; h < kwB; h += TB) {
            stage64x2<T>(sm.S, A + (int64_t)r0 * lda + k0 + h, lda, nr, TB, sm.P, B + (int64_t)(k0 + h) * ldb + c0, ldb,
                         TB, nc);
            __syncthreads();
            acc64_mma<T, true>(acc, [&](int r, int k) { return sm.S[r * LDT + k]; },
                               [&](int k, int c) { return sm.P[k * LDT + c]; });
            __syncthreads();
        }
        acc64_store(acc, C);
        return;
    }
panel:
    /* a panel tile: its own pending update, then the solve against the
     * factored diagonal tile */
    panel_tile(q);
    const int k0 = d0 - kw;
    Acc64<T> acc;
    acc64_load(acc, DenseC<T>{G_, ldg, nr, nc});
    for (int h = 0; h < kw; h += TB) {
        /* tile -= L_{r0,pending} * (U_{pending,c0} or Y_{pending}) */
        if (kind == 2)
            stage64x2<T>(sm.S, A + (int64_t)r0 * lda + k0 + h, lda, nr, TB, sm.P, B + (int64_t)(k0 + h) * ldb + c0, ldb,
                         TB, nc);
        else
            stage64x2<T>(sm.S, A + (int64_t)r0 * lda + k0 + h, lda, nr, TB, sm.P, A + (int64_t)(k0 + h) * lda + c0, lda,
                         TB, nc);
        __syncthreads();
        acc64_mma<T, true>(acc, [&](int r, int k) { return sm.S[r * LDT + k]; },
                           [&](int k, int c) { return sm.P[k * LDT + c]; });
        __syncthreads();
    }
    acc64_store(acc, LdsTile<T>{sm.S});
    __syncthreads();
    /* the solve against the factored diagonal tile, block step p as soon as
     * strip p of its pack is published (its flag counts 3 per strip): each
     * wave keeps its 16-wide slab of the tile in accumulators (transposed for
     * the L tiles, X = A U^{-1} solved as U^T X^T = A^T) and runs step p
     * with the strip staged in P: the diagonal block times the inverse of the
     * strip's diagonal block, then its contribution removed from the blocks
     * after it, each product taking the finished block as its B operand */
    typedef typename vec4<T>::type V;
    const bool right = kind == 1;
    const int w = wave_id(), l = threadIdx.x & 63, lr = l & 15, lk = l >> 4;
    const T *Add = A + (int64_t)d0 * lda + d0;
    V a[4];
#pragma unroll
    for (int q2 = 0; q2 < 4; ++q2)
#pragma unroll
        for (int r = 0; r < 4; ++r)
            a[q2][r] = right ? sm.S[(16 * w + lr) * LDT + 16 * q2 + acc_row<T>(lk, r)]
                             : sm.S[(16 * q2 + acc_row<T>(lk, r)) * LDT + 16 * w + lr];
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        wait_solved(flag, 3 * p + 2, &s_avail, status, wlim);
        /* strip p: rows 16p.. of columns 16p..16p+15 (lower), or columns
         * 16p.. of rows 16p..16p+15 (right); diagonal block from Pg,
         * identity past the matrix end */
        const int len = 64 - 16 * p;
        T v[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int idx = threadIdx.x + NT * i;
            const int r = right ? 16 * p + idx / len : 16 * p + (idx >> 4);
            const int c = right ? 16 * p + idx % len : 16 * p + (idx & 15);
            v[i] = idx >= len * 16 ? T(0)
                   : (r >> 4) == (c >> 4) ? load_coherent(Pg + r * TB + c)
                   : (r < dw && c < dw)   ? load_coherent(Add + (int64_t)r * lda + c)
                                          : T(0);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int idx = threadIdx.x + NT * i;
            const int r = right ? 16 * p + idx / len : 16 * p + (idx >> 4);
            const int c = right ? 16 * p + idx % len : 16 * p + (idx & 15);
            if (idx < len * 16)
                sm.P[r * LDT + c] = v[i];
        }
        __syncthreads();
        V x = {0, 0, 0, 0};
        if (right) {
            wave_mma16_acc<T>(
                x,
                [&](int r, int k) {
                    const T u = sm.P[(16 * p + k) * LDT + 16 * p + r];
                    return k <= r ? u : T(0);
                },
                a[p]);
            a[p] = x;
#pragma unroll
            for (int q2 = p + 1; q2 < 4; ++q2)
                wave_mma16_acc<T>(a[q2], [&](int r, int k) { return -sm.P[(16 * p + k) * LDT + 16 * q2 + r]; }, a[p]);
        } else {
            wave_mma16_acc<T>(
                x,
                [&](int r, int k) {
                    const T u = sm.P[(16 * p + r) * LDT + 16 * p + k];
                    return r > k ? u : (r == k ? T(1) : T(0));
                },
                a[p]);
            a[p] = x;
#pragma unroll
            for (int q2 = p + 1; q2 < 4; ++q2)
                wave_mma16_acc<T>(a[q2], [&](int r, int k) { return -sm.P[(16 * q2 + r) * LDT + 16 * p + k]; }, a[p]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int q2 = 0; q2 < 4; ++q2)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            if (right)
                sm.S[(16 * w + lr) * LDT + 16 * q2 + acc_row<T>(lk, r)] = a[q2][r];
            else
                sm.S[(16 * q2 + acc_row<T>(lk, r)) * LDT + 16 * w + lr] = a[q2][r];
        }
    __syncthreads();
    lds_store_tile(sm.S, G_, ldg, nr, nc);
}

/* ----------------------------------------- update-kernel measurement --- */

/* When enabled on a handle, dense_factor brackets every block-step launch
 * with a pair of events (created up front) and records the launch's
 * algorithmic flop count, so that the caller can report the kernel's live
 * average duration and achieved rate. */
int profile_update_enable(UpdateProfile &p, int max_launches)
{
    for (hipEvent_t e : p.ev)
        (void)hipEventDestroy(e);
    p.ev.clear();
    p.flops.clear();
    p.used = 0;
    if (max_launches <= 0)
        return 0;
    p.ev.resize(2 * (size_t)max_launches);
    p.flops.resize((size_t)max_launches);
    for (hipEvent_t &e : p.ev)
        if (hipEventCreate(&e) != hipSuccess)
            return 1;
    return 0;
}

int profile_update_read(UpdateProfile &p, double *ms_total, int64_t *launches, double *flops_total)
{
    double ms = 0.0, fl = 0.0;
    for (int i = 0; i < p.used; ++i) {
        if (hipEventSynchronize(p.ev[2 * i + 1]) != hipSuccess)
            return 1;
        float t = 0.f;
        if (hipEventElapsedTime(&t, p.ev[2 * i], p.ev[2 * i + 1]) != hipSuccess)
            return 1;
        ms += t;
        fl += p.flops[i];
    }
    *ms_total = ms;
    *launches = p.used;
    *flops_total = fl;
    p.used = 0;
    return 0;
}

static bool profile_slot(UpdateProfile *p, hipStream_t st, double flops, int &slot)
{
    if (!p || p->used >= (int)p->flops.size())
        return false;
    slot = p->used++;
    p->flops[slot] = flops;
    (void)hipEventRecord(p->ev[2 * slot], st);
    return true;
}

/* Launch-per-phase factor: k_diag, then per block step k_panel + k_update. */
template <typename T>
static hipError_t factor_phases(T *A, int64_t lda, int n, int32_t *info, T *Pg, const DenseTuning &tun,
                                UpdateProfile *pr, hipStream_t st, T *B, int64_t ldb, int nrhs)
{
    const int nbc = B ? (nrhs + TB - 1) / TB : 0;
    hipError_t e = hipSuccess;
    hipLaunchKernelGGL(k_diag<T>, dim3(1), dim3(NT), 0, st, A, lda, n, 0, info, Pg, B ? 1 : 0);
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    for (int k0 = 0; k0 < n; k0 += TB) {
        const int kw = min(TB, n - k0);
        const int nrem = (n - k0 - kw + TB - 1) / TB;
        if (nrem == 0 && !B)
            break;
        hipLaunchKernelGGL(k_panel<T>, dim3(2 * nrem + nbc), dim3(NT), 0, st, A, lda, n, k0, Pg, B, ldb, nrhs);
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
        if (nrem == 0)
            break;
        const int m = n - k0 - kw;
        const int nbr = (m + TB - 1) / TB;
        int pslot = -1;
        const bool prof = profile_slot(pr, st, 2.0 * (double)m * (double)m * (double)kw, pslot);
        if (m > tun.small_update_below) {
            const int nt = ((m + 127) / 128) * ((m + 127) / 128);
            hipLaunchKernelGGL((k_update<T, 128, 128, 16>), dim3(nt + 1 + nbr * nbc), dim3(NT), 0, st, A, lda, n,
                               k0, kw, info, Pg, B, ldb, nrhs);
        } else {
            const int nt = ((m + 63) / 64) * ((m + 63) / 64);
            hipLaunchKernelGGL((k_update<T, 64, 64, 16>), dim3(nt + 1 + nbr * nbc), dim3(NT), 0, st, A, lda, n,
                               k0, kw, info, Pg, B, ldb, nrhs);
        }
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
        if (prof)
            (void)hipEventRecord(pr->ev[2 * pslot + 1], st);
    }
    return e;
}

/* Look-ahead factor: one k_step launch per diagonal tile.  While the region
 * past the current panel is large (> tun.defer_above), the block columns are
 * split into G = tun.defer_group classes (J mod G) and launch s updates the
 * region's tiles of class (s + 1) mod G only, with K = 64 G: every tile is
 * read and written once per G steps, every launch carries about the same
 * update work beside the diagonal tile's critical path, and the class of
 * the next diagonal tile is always the one just updated (so the diagonal
 * tile and the L panel apply a single step).  Smaller regions are updated in
 * full in every launch.  applied[c] counts the steps applied to class c. */
template <typename T>
static hipError_t factor_lookahead(T *A, int64_t lda, int n, int32_t *info, T *Pg, int *ctl,
                                   const DenseTuning &tun, UpdateProfile *pr, hipStream_t st, T *B, int64_t ldb,
                                   int nrhs, bool prefilled)
{
    const int nb = (n + TB - 1) / TB;
    const int nbc = B ? (nrhs + TB - 1) / TB : 0;
    const int G = max(1, min(4, sizeof(T) == 4 ? tun.defer_group_f32 : tun.defer_group));
    hipError_t e = hipSuccess;
    (void)prefilled;
    /* workgroups resident at once (two per compute unit), less the diagonal
     * tile's: the size of the first wave of region tiles */
    int dev = 0, cus = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess ||
        (e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
        return e;
    const int first_wave = max(1, 2 * cus - 1);
    const long wlim = tun.wait_limit > 0 ? (long)tun.wait_limit : 1L << 24;
    int applied[4] = {0, 0, 0, 0};
    for (int s = 0; s < nb; ++s) {
        const int d0 = s * TB, e0 = min(n, d0 + TB), m2 = n - e0;
        const int nr2 = (m2 + TB - 1) / TB, J0 = s + 1;
        int pend[4], pendp = 0;
        for (int c = 0; c < 4; ++c) {
            pend[c] = c < G ? s - applied[c] : 0;
            pendp |= pend[c] << (8 * c);
        }
        /* updated classes: none in the first launch, one while split, else all */
        const int upd = s == 0 ? -2 : (G > 1 && m2 > tun.defer_above && s + 1 < nb) ? (s + 1) % G : -1;
        const bool tall = m2 > tun.small_update_below;
        const int bm = tall ? 128 : 64;
        const int jfirst = upd < 0 ? 0 : ((upd - J0 % G) % G + G) % G, jstep = upd < 0 ? 1 : G;
        const int ncu = upd == -2 || jfirst >= nr2 ? 0 : (nr2 - jfirst + jstep - 1) / jstep;
        const int nt2 = ((m2 + bm - 1) / bm) * ncu;
        const int nb2 = s > 0 ? nr2 * nbc : 0;
        const int grid = 1 + nt2 + nb2 + 2 * nr2 + nbc;
        /* algorithmic update flops of the launch: the diagonal tile, the
         * panel tiles and the updated region tiles, 2 rows cols K each */
        const double dw = n - d0 < TB ? n - d0 : TB;
        double fl = 2.0 * dw * dw * TB * pend[s % G];
        for (int j = 0; j < nr2; ++j) {
            const int J = J0 + j;
            const double cols = min(TB, n - (e0 + j * TB));
            const double kwj = (double)TB * pend[J % G];
            fl += 2.0 * dw * cols * kwj;                                    /* U tile (s, J) */
            fl += 2.0 * cols * dw * TB * pend[s % G];                       /* L tile (J, s) */
            if (upd == -1 || (upd >= 0 && J % G == upd))
                fl += 2.0 * m2 * cols * kwj;                                /* region column J */
        }
        int pslot = -1;
        const bool prof = s > 0 && profile_slot(pr, st, fl, pslot);
        if (tall)
            hipLaunchKernelGGL((k_step<T, 128, 64, 16>), dim3(grid), dim3(NT), 0, st, A, lda, n, s, G, upd, pendp,
                               first_wave, info, Pg, B, ldb, nrhs, ctl, wlim);
        else
            hipLaunchKernelGGL((k_step<T, 64, 64, 16>), dim3(grid), dim3(NT), 0, st, A, lda, n, s, G, upd, pendp,
                               first_wave, info, Pg, B, ldb, nrhs, ctl, wlim);
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
        if (prof)
            (void)hipEventRecord(pr->ev[2 * pslot + 1], st);
        if (upd == -1)
            for (int c = 0; c < G; ++c)
                applied[c] = s;
        else if (upd >= 0)
            applied[upd] = s;
    }
    return e;
}

template <typename T>
hipError_t dense_factor(T *A, int64_t lda, int n, int32_t *info, void *ws, const DenseTuning &tun,
                        UpdateProfile *pr, hipStream_t st, T *B, int64_t ldb, int nrhs, bool prefilled)
{
    if (nrhs <= 0)
        B = nullptr;
    if (info && !prefilled) {
        hipError_t e = fill_i32(info, 1, 0, st);
        if (e != hipSuccess)
            return e;
    }
    int *ctl = static_cast<int *>(ws);
    T *Pg = reinterpret_cast<T *>(static_cast<char *>(ws) + factor_ctl_bytes(n));
    if (!prefilled) { /* status word and the block steps' counters */
        hipError_t e = fill_i32(ctl, kCtlHead + 2 * (int64_t)((n + TB - 1) / TB), 0, st);
        if (e != hipSuccess)
            return e;
    }
    if (tun.lookahead)
        return factor_lookahead(A, lda, n, info, Pg, ctl, tun, pr, st, B, ldb, nrhs, prefilled);
    return factor_phases(A, lda, n, info, Pg, tun, pr, st, B, ldb, nrhs);
}

/* Start of a factor + solve: the control words and info cleared and the
 * backward substitution's exchange rows marked unsolved, in one launch. */
template <typename T>
__global__ void k_init_factor_solve(int *ctl, int nctl, int32_t *info, T *xb, int64_t nxb)
{
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, step = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = i0; i < nctl; i += step)
        ctl[i] = 0;
    if (info && i0 == 0)
        *info = 0;
    if (sizeof(T) == 8) {
        unsigned long long *x = reinterpret_cast<unsigned long long *>(xb);
        for (int64_t i = i0; i < nxb; i += step)
            x[i] = kUnsolvedMark64;
    } else {
        unsigned int *x = reinterpret_cast<unsigned int *>(xb);
        for (int64_t i = i0; i < nxb; i += step)
            x[i] = kUnsolvedMark32;
    }
}

template <typename T>
hipError_t factor_solve(T *A, int64_t lda, int n, int32_t *info, void *ws, const DenseTuning &tun, UpdateProfile *pr,
                        hipStream_t st, T *B, int64_t ldb, int nrhs)
{
    const int nb = (n + TB - 1) / TB;
    int *ctl = static_cast<int *>(ws);
    T *xb = reinterpret_cast<T *>(static_cast<char *>(ws) + factor_ws_bytes(sizeof(T), n));
    const int64_t nxb = nrhs > 0 ? (int64_t)(kTrsvHelpers + 1) * nb * TB * 16 : 0;
    const int grid = (int)std::min<int64_t>((nxb + 255) / 256 + 1, 1024);
    hipLaunchKernelGGL((k_init_factor_solve<T>), dim3(grid), dim3(256), 0, st, ctl, kCtlHead + 2 * nb, info, xb, nxb);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess)
        e = dense_factor<T>(A, lda, n, info, ws, tun, pr, st, B, ldb, nrhs, true);
    if (e != hipSuccess)
        return e;
    /* the backward substitution reports the status word into info at its
     * end; without right-hand sides a separate launch does */
    if (nrhs > 0)
        return dense_trsv<T>(TRI_U, A, lda, n, B, ldb, nrhs, ctl, xb, nullptr, info, st, true, tun.wait_limit);
    return fold_status(ctl, info, st);
}

/* ------------------------------------------------- triangular solves --- */

/*
 * Multi-workgroup triangular solve op(T) Y = B (Eq. 1, blocked): per
 * 64-row block, kTrsvHelpers helper workgroups and the block's own, tickets
 * taken in solve order (a block's helpers before it).  The block's own
 * workgroup does everything that does not need the block solved just
 * before it first:
 *   - the inverse of its diagonal operator block D (tile_inv16 on the
 *     factored diagonal tile) and W_j = D^{-1} M_j for the two blocks solved
 *     just before it;
 *   - the contributions of all earlier blocks, as they appear:
 *     r = b - sum_j M_j y_j (the older ones shared with its helpers, whose
 *     partial sums follow the exchange rows, marked like them), and
 *     z = D^{-1} r;
 * so that each of the two last blocks costs one product in registers as it
 * arrives: y = z - W_{j1} y_{j1} - W_{j2} y_{j2} (the two products in an
 * accumulator of their own, so neither waits for z).  Up to 16 right-hand
 * sides per launch (the 16 columns of the matrix-core products); wave w
 * owns rows 16w..16w+15 of the block.
 * Solved blocks are exchanged through XB (n rounded up to 64 rows, pitch 16,
 * filled with the unsolved mark before the launch): a workgroup stores its
 * block there with coherent stores and, without waiting for them, raises
 * the solved-blocks counter.  The workgroups of the next three blocks poll
 * a block's values directly (re-reading until none is the mark), so each of
 * those dependencies costs one round trip; every other reader first waits
 * for the counter to pass the block and reads it through the caches, so the
 * lines being polled see three readers rather than every later workgroup.
 * Solutions also go to B.
 */
template <typename T, int MODE>
__global__ __launch_bounds__(NT) void k_trsv(const T *__restrict__ LU, int64_t lda, int n, T *__restrict__ B,
                                             int64_t ldb, int nrhs_here, int *wsi, T *__restrict__ XB, const int *skip,
                                             int32_t *info, long wlim)
{
    typedef typename vec4<T>::type V;
    if (skip && *skip)
        return;
    __shared__ TileSmem<T> sm;
    __shared__ T wls[2][16][NT]; /* -W of the last two blocks, A-operand order per thread */
    int *status = wsi, *ctr = wsi + 1, *solved = wsi + 2;
    if (threadIdx.x == 0) {
        sm.ticket = atomicAdd(ctr, 1);
        sm.avail = 0;
    }
    __syncthreads();
    const int nb = (n + TB - 1) / TB;
    if (sm.ticket >= (kTrsvHelpers + 1) * nb) { /* counter not reset: refuse rather than index out of range */
        if (threadIdx.x == 0)
            atomicOr(status, 2);
        return;
    }
    constexpr bool FWD = tri_forward(MODE), TR = tri_trans(MODE), UNITL = (MODE == TRI_L || MODE == TRI_LT);
    /* kTrsvHelpers helpers, then the block's own workgroup, per position:
     * a workgroup only ever waits for lower tickets */
    const int pos = sm.ticket / (kTrsvHelpers + 1), role = sm.ticket % (kTrsvHelpers + 1);
    const bool helper = role < kTrsvHelpers;
    const int blk = FWD ? pos : nb - 1 - pos;
    const int ndep = pos; /* blocks solved before this one */
    const int t = threadIdx.x, w = wave_id(), l = t & 63, lr = l & 15, lk = l >> 4;
    const int r0 = blk * TB, nr = min(TB, n - r0);
    auto dep_blk = [&](int d) { return FWD ? d : nb - 1 - d; };
    /* element (r, k) of operator block (blk, bj): op(T)[r0 + r][bj*64 + k];
     * the address is clamped and the value selected, so the loads of a tile
     * are issued without branches (the compiler then waits for exactly the
     * loads a use needs) */
    auto opel = [&](int bj, int r, int k) -> T {
        const int gr = r0 + r, gk = bj * TB + k;
        const int cr = min(gr, n - 1), ck = min(gk, n - 1);
        const T v = TR ? LU[(int64_t)ck * lda + cr] : LU[(int64_t)cr * lda + ck];
        return ((gr < n) & (gk < n)) ? v : T(0);
    };
    /* this lane's 16 elements of operator block (blk, bj) as the A operand,
     * loaded raw from clamped addresses; a_op applies the bounds where the
     * values are used, so nothing waits for these loads before then */
    auto load_a = [&](int bj, T(&a)[16]) {
        const int cr = min(r0 + 16 * w + lr, n - 1);
#pragma unroll
        for (int ks = 0; ks < 16; ++ks) {
            const int ck = min(bj * TB + 4 * ks + lk, n - 1);
            a[ks] = TR ? LU[(int64_t)ck * lda + cr] : LU[(int64_t)cr * lda + ck];
        }
    };
    auto a_op = [&](int bj, int ks, T a) {
        return ((r0 + 16 * w + lr < n) & (bj * TB + 4 * ks + lk < n)) ? a : T(0);
    };
    /* solved block bj (all 64 rows, as the B operand); every row and column
     * of an exchange block is written by its producer (zeros past n and past
     * the right-hand sides), so the loads need no bounds */
    auto fetch_y = [&](int bj, T(&y)[16]) {
#pragma unroll
        for (int ks = 0; ks < 16; ++ks)
            y[ks] = load_coherent(XB + (int64_t)(bj * TB + 4 * ks + lk) * 16 + lr);
    };
    /* the same through the caches, for a block the counter has passed: the
     * XCD's L2 fetches it once for all its readers instead of every wave of
     * every later workgroup going to the point of coherence.  A cached line
     * can only hold final values or the mark (each element is written once
     * per launch), and a mark sends the reader to load_y's coherent reads. */
    auto fetch_y_cached = [&](int bj, T(&y)[16]) {
#pragma unroll
        for (int ks = 0; ks < 16; ++ks)
            y[ks] = XB[(int64_t)(bj * TB + 4 * ks + lk) * 16 + lr];
    };
    auto has_mark = [&](const T(&y)[16]) {
        bool miss = false;
#pragma unroll
        for (int ks = 0; ks < 16; ++ks)
            miss = miss || is_unsolved_mark(y[ks]);
        return miss;
    };
    /* re-read block bj while any value this wave needs still holds the mark */
    auto load_y = [&](int bj, T(&y)[16]) {
        for (long spins = 0;; ++spins) {
            fetch_y(bj, y);
            if (!__any(has_mark(y)))
                break;
            if (wait_give_up(status, spins, wlim))
                break;
            __builtin_amdgcn_s_sleep(1);
        }
    };

    /* Contributions of the blocks solved before, all but the last three:
     * dependency d goes to role d mod (kTrsvHelpers + 1), so that a block's
     * older dependencies are taken by kTrsvHelpers helper workgroups and its
     * own workgroup together.  One pass per dependency: its values are
     * requested first, then the operator block of this role's next one, so
     * the operator loads overlap the wait for the values; the two operator
     * register sets (and two accumulators) alternate between passes, so no
     * copy makes a pass wait for the loads it has just issued.  The loads are
     * issued unconditionally (indices clamped) so that the waits count only
     * the loads each use needs. */
    constexpr int STRIDE = kTrsvHelpers + 1;
    const int K = ndep - 2;  /* blocks before the last two */
    const int KP = K - 1;    /* ... of which those taken in passes; block K-1 is polled */
    V acc = {0, 0, 0, 0}, acc2 = {0, 0, 0, 0};
    auto pass = [&](int d, const T(&cur)[16], T(&nxt)[16], V &ac) __attribute__((always_inline)) {
        /* read once the counter has passed the block (the values are then
         * normally there: re-read below if not) */
        wait_solved(solved, d, &sm.avail, status, wlim);
        T y[16];
        fetch_y_cached(dep_blk(d), y);
        __builtin_amdgcn_sched_barrier(0);
        load_a(dep_blk(min(d + STRIDE, KP - 1)), nxt);
        __builtin_amdgcn_sched_barrier(0);
        if (__any(has_mark(y)))
            load_y(dep_blk(d), y);
        const int bd = dep_blk(d);
#pragma unroll
        for (int ks = 0; ks < 16; ++ks)
            ac = mfma16(a_op(bd, ks, cur[ks]), y[ks], ac);
    };
    auto passes = [&]() __attribute__((always_inline)) {
        if (role < KP) {
            T a0[16], a1[16];
            load_a(dep_blk(role), a0);
            for (int d = role; d < KP; d += 2 * STRIDE) {
                pass(d, a0, a1, acc);
                if (d + STRIDE < KP)
                    pass(d + STRIDE, a1, a0, acc2);
            }
        }
    };
    /* the helpers' partial sums follow the exchange rows, in accumulator
     * layout (thread t's four values at 4t), marked like them */
    T *PB = XB + (int64_t)nb * TB * 16;
    if (helper) {
        passes();
        T *pp = PB + ((int64_t)pos * kTrsvHelpers + role) * (TB * 16) + 4 * t;
#pragma unroll
        for (int r = 0; r < 4; ++r)
            store_coherent(pp + r, acc[r] + acc2[r]);
        return;
    }

    /* own right-hand side, in accumulator layout (rows 16w + acc_row, column lr) */
    V rhs;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = 16 * w + acc_row<T>(lk, r);
        rhs[r] = (row < nr && lr < nrhs_here) ? B[(int64_t)(r0 + row) * ldb + lr] : T(0);
    }

    /* inverse of the diagonal operator block, from the factored tile; it
     * stays in sm.t1 and is read into registers where it is used */
    stage_tile_identity(sm.t0, LU + (int64_t)r0 * lda + r0, lda, nr, nr);
    __syncthreads();
    if (t < TB)
        sm.rinv[t] = recip(sm.t0[t * (LDT + 1)]);
    __syncthreads();
    tile_inv16(sm.t0, sm.rinv, sm.t1);
    auto load_dinv = [&](T(&dA)[16]) { /* op(D)^{-1}[16w + lr][4ks + lk] */
#pragma unroll
        for (int ks = 0; ks < 16; ++ks) {
            const int r = 16 * w + lr, k = 4 * ks + lk;
            const int i = TR ? k : r, j = TR ? r : k; /* element (i, j) of L^{-1} or U^{-1} */
            const T v = sm.t1[i * LDT + j];
            dA[ks] = UNITL ? (i > j ? v : (i == j ? T(1) : T(0))) : (i <= j ? v : T(0));
        }
    };

    /* -W_j = -D^{-1} M_j for the two blocks solved last (M_j: their operator
     * blocks), needed only after the last waits but independent of every
     * solution: formed now and kept in LDS in this thread's A-operand order */
    auto form_w = [&](int bj, const T(&dA)[16], int slot) {
        tile_xfer<T>([&](int r, int c) { return opel(bj, r, c); }, [&](int r, int c, T v) { sm.t0[r * LDT + c] = v; });
        __syncthreads();
        V wacc[4];
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
            wacc[cb] = V{0, 0, 0, 0};
#pragma unroll
            for (int ks = 0; ks < 16; ++ks)
                wacc[cb] = mfma16(dA[ks], sm.t0[(4 * ks + lk) * LDT + 16 * cb + lr], wacc[cb]);
        }
        __syncthreads();
#pragma unroll
        for (int cb = 0; cb < 4; ++cb)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                sm.t0[(16 * w + acc_row<T>(lk, r)) * LDT + 16 * cb + lr] = wacc[cb][r];
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < 16; ++ks)
            wls[slot][ks][t] = -sm.t0[(16 * w + lr) * LDT + 4 * ks + lk];
        __syncthreads();
    };
    {
        T dA[16];
        load_dinv(dA);
        if (ndep >= 1)
            form_w(dep_blk(ndep - 1), dA, 0);
        if (ndep >= 2)
            form_w(dep_blk(ndep - 2), dA, 1);
    }

    if (K > 0) {
        T al[16]; /* operator block of block K-1, loaded first */
        load_a(dep_blk(K - 1), al);
        passes();
        /* block K-1 (three before this one) is polled directly: at the front
         * of the chain it is what z waits for */
        T y[16];
        load_y(dep_blk(K - 1), y);
        const int bl = dep_blk(K - 1);
#pragma unroll
        for (int ks = 0; ks < 16; ++ks)
            acc = mfma16(a_op(bl, ks, al[ks]), y[ks], acc);
        /* the helpers' partial sums, re-read until none is the mark */
#pragma unroll
        for (int h = 0; h < kTrsvHelpers; ++h) {
            const T *pp = PB + ((int64_t)pos * kTrsvHelpers + h) * (TB * 16) + 4 * t;
            T pv[4];
            for (long spins = 0;; ++spins) {
                bool miss = false;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    pv[r] = load_coherent(pp + r);
                    miss = miss || is_unsolved_mark(pv[r]);
                }
                if (!__any(miss))
                    break;
                if (wait_give_up(status, spins, wlim))
                    break;
                __builtin_amdgcn_s_sleep(1);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r)
                acc[r] += pv[r];
        }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
        acc[r] += acc2[r];

    /* x = D^{-1} (b - acc), through LDS (rows of r come from all four waves),
     * then - W_j y_j for the two blocks solved last, each a product in
     * registers as its values arrive */
    T *Rl = sm.t0; /* 64 x 16, pitch 17 */
#pragma unroll
    for (int r = 0; r < 4; ++r)
        Rl[(16 * w + acc_row<T>(lk, r)) * 17 + lr] = rhs[r] - acc[r];
    __syncthreads();
    V x = {0, 0, 0, 0};
    {
        T dA[16];
        load_dinv(dA);
#pragma unroll
        for (int ks = 0; ks < 16; ++ks)
            x = mfma16(dA[ks], Rl[(4 * ks + lk) * 17 + lr], x);
    }
    /* the last two blocks, polled directly, into their own accumulator so
     * that neither waits for z */
    V xw = {0, 0, 0, 0};
    if (ndep >= 2) {
        T wa[16], y[16];
#pragma unroll
        for (int ks = 0; ks < 16; ++ks)
            wa[ks] = wls[1][ks][t];
        load_y(dep_blk(ndep - 2), y);
#pragma unroll
        for (int ks = 0; ks < 16; ++ks)
            xw = mfma16(wa[ks], y[ks], xw);
    }
    if (ndep >= 1) {
        T wa[16], y[16];
#pragma unroll
        for (int ks = 0; ks < 16; ++ks)
            wa[ks] = wls[0][ks][t];
        load_y(dep_blk(ndep - 1), y);
#pragma unroll
        for (int ks = 0; ks < 16; ++ks)
            xw = mfma16(wa[ks], y[ks], xw);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
        x[r] += xw[r];
    /* all 64 rows and 16 columns of the exchange block are written (zeros
     * outside the system), the solution rows also to B */
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = 16 * w + acc_row<T>(lk, r);
        const bool ok = row < nr && lr < nrhs_here;
        store_coherent(XB + (int64_t)(r0 + row) * 16 + lr, ok ? x[r] : T(0));
        if (ok)
            B[(int64_t)(r0 + row) * ldb + lr] = x[r];
    }
    /* the hint for the readers of later blocks (they check the values); a
     * maximum, since without a wait for the stores above the updates of
     * consecutive blocks may land out of order */
    __syncthreads();
    if (t == 0)
        __hip_atomic_fetch_max(solved, pos + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    /* the last block's workgroup ends after every wait of the launch has
     * ended (each block waited for the one before it and for its helpers),
     * so a give-up anywhere is in the status word by now: report it */
    if (info && pos == nb - 1 && t == 0) {
        __threadfence();
        const int st = load_coherent(status);
        if (st)
            *info = -st;
    }
}

template <typename T, int MODE>
static hipError_t trsv_mode(const T *LU, int64_t lda, int n, T *B, int64_t ldb, int nrhs, int *wsi, T *xb,
                            const int *skip, int32_t *info, hipStream_t st, bool prefilled, long wlim)
{
    const int nb = (n + TB - 1) / TB;
    hipError_t e = hipSuccess;
    for (int c0 = 0; c0 < nrhs; c0 += 16) {
        const int nh = min(16, nrhs - c0);
        if (!(prefilled && c0 == 0)) { /* counters cleared, exchange rows marked */
            if ((e = fill_i32(wsi + 1, kCtlHead - 1, 0, st)) != hipSuccess)
                return e;
            if ((e = fill_unsolved(xb, (int64_t)(kTrsvHelpers + 1) * nb * TB * 16, st)) != hipSuccess)
                return e;
        }
        hipLaunchKernelGGL((k_trsv<T, MODE>), dim3((kTrsvHelpers + 1) * nb), dim3(NT), 0, st, LU, lda, n, B + c0, ldb,
                           nh, wsi, xb, skip, info, wlim);
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
    }
    return e;
}

template <typename T>
hipError_t dense_trsv(int mode, const T *LU, int64_t lda, int n, T *B, int64_t ldb, int nrhs, int *wsi, T *xb,
                      const int *skip, int32_t *info, hipStream_t st, bool prefilled, long long wait_limit)
{
    const long wl = wait_limit > 0 ? (long)wait_limit : 1L << 22;
    switch (mode) {
    case TRI_L: return trsv_mode<T, TRI_L>(LU, lda, n, B, ldb, nrhs, wsi, xb, skip, info, st, prefilled, wl);
    case TRI_U: return trsv_mode<T, TRI_U>(LU, lda, n, B, ldb, nrhs, wsi, xb, skip, info, st, prefilled, wl);
    case TRI_UT: return trsv_mode<T, TRI_UT>(LU, lda, n, B, ldb, nrhs, wsi, xb, skip, info, st, prefilled, wl);
    default: return trsv_mode<T, TRI_LT>(LU, lda, n, B, ldb, nrhs, wsi, xb, skip, info, st, prefilled, wl);
    }
}

/* ---------------------------------------------------- uniform batches --- */

template <typename T>
__global__ __launch_bounds__(NT, 2) void k_lu_batch(T *__restrict__ A, int64_t lda, int n, int64_t strideA,
                                                    int32_t *info)
{
    __shared__ TileSmem<T> sm;
    T *Ab = A + (int64_t)blockIdx.x * strideA;
    const int z = wg_crout<T>(Ab, lda, n, nullptr, 0, 0, sm);
    if (threadIdx.x == 0 && info)
        info[blockIdx.x] = z;
}

template <typename T, int M1, int M2, int NR>
__global__ __launch_bounds__(NT, 2) void k_solve_batch(const T *__restrict__ LU, int64_t lda, int n, int64_t strideLU,
                                                       T *__restrict__ B, int64_t ldb, int64_t strideB, int nrhs_here)
{
    __shared__ TileSmem<T> sm;
    const T *L = LU + (int64_t)blockIdx.x * strideLU;
    T *Bb = B + (int64_t)blockIdx.x * strideB;
    wg_solve<T, M1, NR>(L, lda, n, Bb, ldb, nrhs_here, sm);
    wg_solve<T, M2, NR>(L, lda, n, Bb, ldb, nrhs_here, sm);
}

/* One right-hand side per system (n <= 64 LDT): both substitutions with the
 * vector in LDS, the factor read once with coalesced loads (wg_trsv1). */
template <typename T, int M1, int M2>
__global__ __launch_bounds__(NT, 2) void k_solve_batch1(const T *__restrict__ LU, int64_t lda, int n, int64_t strideLU,
                                                        T *__restrict__ B, int64_t ldb, int64_t strideB)
{
    __shared__ TileSmem<T> sm;
    const T *L = LU + (int64_t)blockIdx.x * strideLU;
    T *Bb = B + (int64_t)blockIdx.x * strideB;
    for (int i = threadIdx.x; i < n; i += NT)
        sm.t1[i] = Bb[(int64_t)i * ldb];
    __syncthreads();
    wg_trsv1<T, M1>(L, lda, n, sm.t1, sm.t0);
    wg_trsv1<T, M2>(L, lda, n, sm.t1, sm.t0);
    for (int i = threadIdx.x; i < n; i += NT)
        Bb[(int64_t)i * ldb] = sm.t1[i];
}

template <typename T>
hipError_t batch_factor(T *A, int64_t lda, int n, int64_t batch, int64_t strideA, int32_t *info, hipStream_t st)
{
    for (int64_t b0 = 0; b0 < batch; b0 += 65535) {
        const int nb = (int)std::min<int64_t>(65535, batch - b0);
        hipLaunchKernelGGL(k_lu_batch<T>, dim3(nb), dim3(NT), 0, st, A + b0 * strideA, lda, n, strideA,
                           info ? info + b0 : nullptr);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

template <typename T, int M1, int M2>
static hipError_t batch_solve_modes(const T *LU, int64_t lda, int n, int64_t strideLU, T *B, int64_t ldb,
                                    int64_t strideB, int nrhs, int64_t batch, hipStream_t st)
{
    for (int64_t b0 = 0; b0 < batch; b0 += 65535) {
        const int nb = (int)std::min<int64_t>(65535, batch - b0);
        for (int c0 = 0; c0 < nrhs; c0 += 8) {
            const int nh = min(8, nrhs - c0);
            const T *L = LU + b0 * strideLU;
            T *Bb = B + b0 * strideB + c0;
            if (nh == 1 && n <= TB * LDT)
                hipLaunchKernelGGL((k_solve_batch1<T, M1, M2>), dim3(nb), dim3(NT), 0, st, L, lda, n, strideLU, Bb, ldb,
                                   strideB);
            else if (nh == 1)
                hipLaunchKernelGGL((k_solve_batch<T, M1, M2, 1>), dim3(nb), dim3(NT), 0, st, L, lda, n, strideLU, Bb, ldb, strideB, nh);
            else if (nh <= 4)
                hipLaunchKernelGGL((k_solve_batch<T, M1, M2, 4>), dim3(nb), dim3(NT), 0, st, L, lda, n, strideLU, Bb, ldb, strideB, nh);
            else
                hipLaunchKernelGGL((k_solve_batch<T, M1, M2, 8>), dim3(nb), dim3(NT), 0, st, L, lda, n, strideLU, Bb, ldb, strideB, nh);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess)
                return e;
        }
    }
    return hipSuccess;
}

template <typename T>
hipError_t batch_solve(bool adjoint, const T *LU, int64_t lda, int n, int64_t strideLU, T *B, int64_t ldb,
                       int64_t strideB, int nrhs, int64_t batch, hipStream_t st)
{
    if (adjoint)
        return batch_solve_modes<T, TRI_UT, TRI_LT>(LU, lda, n, strideLU, B, ldb, strideB, nrhs, batch, st);
    return batch_solve_modes<T, TRI_L, TRI_U>(LU, lda, n, strideLU, B, ldb, strideB, nrhs, batch, st);
}

/* ----------------------------------------------------- ragged batches --- */

/* Persistent factor + solve of a ragged batch: each workgroup repeatedly
 * takes the next system from the queue (in `order`, the EbV schedule), and
 * factors and solves it alone.  Every workgroup leaves the loop once the
 * queue is exhausted. */
template <typename T>
__global__ __launch_bounds__(NT, 2) void k_batched(int count, const int *__restrict__ ns, const int64_t *__restrict__ offA,
                                                   T *__restrict__ A, const int64_t *__restrict__ offB, T *__restrict__ B,
                                                   const int *__restrict__ order, int32_t *info, int *queue)
{
    __shared__ TileSmem<T> sm;
    for (;;) {
        if (threadIdx.x == 0)
            sm.ticket = atomicAdd(queue, 1);
        __syncthreads();
        /* uniform across the workgroup: the system's addresses stay scalar */
        const int idx = __builtin_amdgcn_readfirstlane(sm.ticket);
        __syncthreads();
        if (idx >= count)
            break;
        const int s = order ? order[idx] : idx;
        const int n = ns[s];
        if (n <= 0 || (int64_t)n * n * (int64_t)sizeof(T) >= kWgMaxSystemBytes) {
            /* empty, or beyond what one workgroup addresses: reported, untouched */
            if (threadIdx.x == 0 && info)
                info[s] = n <= 0 ? 0 : -3;
            continue;
        }
        T *As = A + offA[s];
        T *Bs = B ? B + offB[s] : nullptr;
        /* factor with the forward substitution riding along, then the
         * backward substitution */
        const int z = wg_crout<T>(As, n, n, Bs, 1, 1, sm);
        if (threadIdx.x == 0 && info)
            info[s] = z;
        if (Bs) {
            if (n <= TB * LDT) {
                /* the vector in LDS (sm.t1), the diagonal blocks staged in sm.t0 */
                for (int i = threadIdx.x; i < n; i += NT)
                    sm.t1[i] = Bs[i];
                __syncthreads();
                wg_trsv1<T, TRI_U>(As, n, n, sm.t1, sm.t0);
                for (int i = threadIdx.x; i < n; i += NT)
                    Bs[i] = sm.t1[i];
            } else {
                wg_solve<T, TRI_U, 1>(As, n, n, Bs, 1, 1, sm);
            }
        }
    }
}

/* Largest system whose refinement keeps its vectors in LDS (the float
 * vector in a tile buffer of TileSmem<float>, x in double beside it). */
constexpr int kMixLdsN = TB * LDT;

/* Workgroup-wide maximum (result valid in every thread). */
__device__ double wg_max(double v, double *red)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v = fmax(v, __shfl_xor(v, o));
    __syncthreads();
    if ((threadIdx.x & 63) == 0)
        red[threadIdx.x >> 6] = v;
    __syncthreads();
    v = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    __syncthreads();
    return v;
}

/* Ragged batch, mixed precision: per system a float copy is factored and the
 * float solve is refined in double (residual r = b - A x over the double A,
 * update x += solve_float(r)).  The stop test bounds the forward error: with
 * the system's dominance margin m = min_i (|a_ii| - sum_{j != i} |a_ij|) > 0,
 * ||x - x*||_inf <= ||r||_inf / m, and the loop ends once
 * ||r||_inf <= tol m ||x||_inf (never for m = 0: iters reports -1). */
__global__ __launch_bounds__(NT, 2) void k_batched_mixed(int count, const int *__restrict__ ns, const int64_t *__restrict__ offA,
                                                         const double *__restrict__ A, const int64_t *__restrict__ offB,
                                                         double *__restrict__ B, const int *__restrict__ order,
                                                         int32_t *info, int *queue, float *__restrict__ W,
                                                         float *__restrict__ R32, double *__restrict__ X,
                                                         int max_iter, double tol, int32_t *iters)
{
    __shared__ TileSmem<float> sm;
    __shared__ double xd[kMixLdsN]; /* x in double while the vectors fit LDS */
    __shared__ double red[4];
    const int t = threadIdx.x, w = wave_id(), l = t & 63;
    for (;;) {
        if (t == 0)
            sm.ticket = atomicAdd(queue, 1);
        __syncthreads();
        const int idx = __builtin_amdgcn_readfirstlane(sm.ticket);
        __syncthreads();
        if (idx >= count)
            break;
        const int s = order ? order[idx] : idx;
        const int n = ns[s];
        if (n <= 0 || (int64_t)n * n * (int64_t)sizeof(double) >= kWgMaxSystemBytes) {
            /* empty, or beyond what one workgroup addresses: reported, untouched */
            if (t == 0) {
                if (info)
                    info[s] = n <= 0 ? 0 : -3;
                if (iters)
                    iters[s] = n <= 0 ? 0 : -1;
            }
            continue;
        }
        const double *As = A + offA[s];
        double *bs = B + offB[s];
        float *Ws = W + offA[s];
        float *rs = R32 + offB[s];
        double *xs = X + offB[s];
        /* float copy and dominance margin: wave w takes rows 4w .. 4w+3,
         * 4w+16 .., four rows at a time, its lanes the columns (all of a
         * group's loads issued before its sums) */
        double mrow = __longlong_as_double(0x7FF0000000000000ll);
        const int ngr = 4 * w < n ? (n - 4 * w + 15) / 16 : 0; /* this wave's groups of rows */
        auto grow = [&](int g) { return 4 * w + 16 * g; };
        {
            double off[4] = {0.0, 0.0, 0.0, 0.0}, dg[4] = {0.0, 0.0, 0.0, 0.0};
            wave_rows4_stream<double>(
                As, n, ngr, grow, n, 0, n,
                [&](int g, int cb, const double(&v)[4][4]) {
                    const int i0 = grow(g);
#pragma unroll
                    for (int u = 0; u < 4; ++u)
#pragma unroll
                        for (int m = 0; m < 4; ++m) {
                            const int c = cb + 64 * m + l;
                            if (c < n && i0 + u < n) {
                                Ws[(int64_t)(i0 + u) * n + c] = (float)v[u][m];
                                if (c == i0 + u)
                                    dg[u] = fabs(v[u][m]);
                                else
                                    off[u] += fabs(v[u][m]);
                            }
                        }
                },
                [&](int g) {
                    const int i0 = grow(g);
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
#pragma unroll
                        for (int o = 32; o > 0; o >>= 1) {
                            off[u] += __shfl_xor(off[u], o);
                            dg[u] += __shfl_xor(dg[u], o);
                        }
                        if (i0 + u < n)
                            mrow = fmin(mrow, fmax(dg[u] - off[u], 0.0));
                        off[u] = dg[u] = 0.0;
                    }
                });
        }
        const double margin = -wg_max(-mrow, red);
        for (int i = t; i < n; i += NT)
            rs[i] = (float)bs[i];
        __syncthreads();
        /* float factor with the first forward substitution riding along */
        const int z = wg_crout<float>(Ws, n, n, rs, 1, 1, sm);
        if (t == 0 && info)
            info[s] = z;
        int used = -1;
        if (n <= kMixLdsN) {
            /* vectors in LDS: the float correction (sm.t1) and x in double */
            float *xf = sm.t1;
            for (int i = t; i < n; i += NT)
                xf[i] = rs[i];
            __syncthreads();
            wg_trsv1<float, TRI_U>(Ws, n, n, xf, sm.t0);
            double xmax = 0.0;
            for (int i = t; i < n; i += NT) {
                xd[i] = (double)xf[i];
                xmax = fmax(xmax, fabs(xd[i]));
            }
            xmax = wg_max(xmax, red);
            for (int it = 0;; ++it) {
                /* r = b - A x in double (four rows per wave at a time), kept
                 * in float as the next correction's right-hand side */
                double rmax = 0.0;
                {
                    double sum[4] = {0.0, 0.0, 0.0, 0.0};
                    wave_rows4_stream<double>(
                        As, n, ngr, grow, n, 0, n,
                        [&](int, int cb, const double(&v)[4][4]) {
                            double xv[4];
#pragma unroll
                            for (int m = 0; m < 4; ++m) {
                                const int c = cb + 64 * m + l;
                                xv[m] = c < n ? xd[c] : 0.0;
                            }
#pragma unroll
                            for (int u = 0; u < 4; ++u)
#pragma unroll
                                for (int m = 0; m < 4; ++m)
                                    sum[u] = __builtin_fma(v[u][m], xv[m], sum[u]);
                        },
                        [&](int g) {
                            const int i0 = grow(g);
#pragma unroll
                            for (int u = 0; u < 4; ++u) {
#pragma unroll
                                for (int o = 32; o > 0; o >>= 1)
                                    sum[u] += __shfl_xor(sum[u], o);
                                if (i0 + u < n) {
                                    const double r = bs[i0 + u] - sum[u];
                                    rmax = fmax(rmax, fabs(r));
                                    if (l == 0)
                                        xf[i0 + u] = (float)r;
                                }
                                sum[u] = 0.0;
                            }
                        });
                }
                rmax = wg_max(rmax, red);
                if (rmax == 0.0 || rmax <= tol * margin * xmax) {
                    used = it;
                    break;
                }
                if (it == max_iter)
                    break;
                /* d = solve_float(r), x += d */
                wg_trsv1<float, TRI_L>(Ws, n, n, xf, sm.t0);
                wg_trsv1<float, TRI_U>(Ws, n, n, xf, sm.t0);
                xmax = 0.0;
                for (int i = t; i < n; i += NT) {
                    xd[i] += (double)xf[i];
                    xmax = fmax(xmax, fabs(xd[i]));
                }
                xmax = wg_max(xmax, red);
            }
            __syncthreads();
            for (int i = t; i < n; i += NT)
                bs[i] = xd[i];
        } else {
            for (int it = 0; it <= max_iter; ++it) {
                if (it > 0)
                    wg_solve<float, TRI_L, 1>(Ws, n, n, rs, 1, 1, sm);
                wg_solve<float, TRI_U, 1>(Ws, n, n, rs, 1, 1, sm);
                double xmax = 0.0;
                for (int i = t; i < n; i += NT) {
                    const double x = (it == 0) ? (double)rs[i] : xs[i] + (double)rs[i];
                    xs[i] = x;
                    xmax = fmax(xmax, fabs(x));
                }
                xmax = wg_max(xmax, red);
                __syncthreads();
                /* r = b - A x: wave w takes rows w, w+4, ...; lanes split the row */
                double rmax = 0.0;
                for (int i = w; i < n; i += 4) {
                    double sacc = 0.0;
                    for (int j = l; j < n; j += 64)
                        sacc += As[(int64_t)i * n + j] * xs[j];
#pragma unroll
                    for (int o = 32; o > 0; o >>= 1)
                        sacc += __shfl_xor(sacc, o);
                    const double r = bs[i] - sacc;
                    if (l == 0)
                        rs[i] = (float)r;
                    rmax = fmax(rmax, fabs(r));
                }
                rmax = wg_max(rmax, red);
                if (rmax == 0.0 || rmax <= tol * margin * xmax) {
                    used = it;
                    break;
                }
            }
            __syncthreads();
            for (int i = t; i < n; i += NT)
                bs[i] = xs[i];
        }
        if (t == 0 && iters)
            iters[s] = used;
        __syncthreads();
    }
}

template <typename T>
hipError_t batched_run(int count, const int *ns, const int64_t *offA, T *A, const int64_t *offB, T *B,
                       const int *order, int32_t *info, int *queue, int grid, hipStream_t st)
{
    hipError_t e = fill_i32(queue, 1, 0, st);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_batched<T>, dim3(grid), dim3(NT), 0, st, count, ns, offA, A, offB, B, order, info, queue);
    return hipGetLastError();
}

hipError_t batched_mixed_run(int count, const int *ns, const int64_t *offA, const double *A, const int64_t *offB,
                             double *B, const int *order, int32_t *info, int *queue, float *W, float *R32,
                             double *X, int max_iter, double tol, int32_t *iters, int grid, hipStream_t st)
{
    hipError_t e = fill_i32(queue, 1, 0, st);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_batched_mixed, dim3(grid), dim3(NT), 0, st, count, ns, offA, A, offB, B, order, info, queue,
                       W, R32, X, max_iter, tol, iters);
    return hipGetLastError();
}

/* ---------------------------------------------------------------- band --- */

/*
 * Tile (rb, cb) of a band matrix in row-wise band storage (a_ij at
 * AB[i*ldab + j - i + kl] for -kl <= j - i <= ku): element (r, c) is
 * a_{64rb+r, 64cb+c}, held in slot c - r + d0 of storage row 64rb + r with
 * d0 = 64 (cb - rb) + kl.  It exists when that slot lies in 0..kl+ku and its
 * row and column are inside the matrix.  Loads are unconditional (`raw`: the
 * tile's first slot stands in for an element that does not exist, and the
 * user masks with `in`), so that a run of them stays in flight together
 * instead of each waiting behind a branch.
 */
struct BandTile {
    double *base; /* storage row 64 rb */
    int64_t ldab;
    int d0, w, nr, nc;
    __device__ __forceinline__ BandTile(double *AB, int64_t ldab_, int n, int kl, int ku, int rb, int cb)
        : base(AB + (int64_t)rb * TB * ldab_), ldab(ldab_), d0(TB * (cb - rb) + kl), w(kl + ku), nr(n - TB * rb),
          nc(n - TB * cb)
    {
    }
    __device__ __forceinline__ bool in(int r, int c) const
    {
        return (unsigned)(c - r + d0) <= (unsigned)w && r < nr && c < nc;
    }
    __device__ __forceinline__ double *addr(int r, int c) const { return base + (int64_t)r * ldab + (c - r + d0); }
    __device__ __forceinline__ double raw(int r, int c) const { return *(in(r, c) ? addr(r, c) : base); }
    /* accumulator address map (acc64_store): nullptr where no element */
    __device__ __forceinline__ double *operator()(int r, int c) const { return in(r, c) ? addr(r, c) : nullptr; }
};

/* LDS of the band factor: the running diagonal tile and the tiles right of it
 * and below it. */
struct BandSmem {
    double s[TB * LDT];
    double u[TB * LDT];
    double l[TB * LDT];
    double rinv[TB];
    double aux[32 + 256];
    int zflag;
};

/*
 * One 16-wide panel q of the band step's off-diagonal tiles, by one wave,
 * once panel q of the diagonal tile S is factored (tile_lu16): U = the tile
 * right of S, L = the tile below it (LDS, pitch LDT).
 *   UPPER: rows 16q.. of U become U_{k,k+1}'s: L_qq^{-1} applied by forward
 *     substitution (lane = column, the unit-lower coefficients read from S
 *     as broadcasts), then the panel's rank-16 term leaves the rows below;
 *   else:  columns 16q.. of L become L_{k+1,k}'s: U_qq^{-1} applied from the
 *     right (lane = row), then the panel's rank-16 term leaves the columns
 *     to the right.
 */
template <bool UPPER>
__device__ __forceinline__ void band_panel(const double *S, const double *rinv, double *X, int q)
{
    typedef vec4<double>::type V;
    const int lane = launder((int)threadIdx.x & 63), c0 = 16 * q;
    S = launder(S);
    X = launder(X);
    double x[16];
    if (UPPER) {
#pragma unroll
        for (int i = 0; i < 16; ++i)
            x[i] = X[(c0 + i) * LDT + lane];
#pragma unroll
        for (int kk = 0; kk < 15; ++kk) {
#pragma unroll
            for (int i = kk + 1; i < 16; ++i)
                x[i] = __builtin_fma(-S[(c0 + i) * LDT + c0 + kk], x[kk], x[i]);
            pin16(x);
        }
#pragma unroll
        for (int i = 0; i < 16; ++i)
            X[(c0 + i) * LDT + lane] = x[i];
    } else {
#pragma unroll
        for (int j = 0; j < 16; ++j)
            x[j] = X[lane * LDT + c0 + j];
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            x[j] *= rinv[c0 + j];
#pragma unroll
            for (int jj = j + 1; jj < 16; ++jj)
                x[jj] = __builtin_fma(-S[(c0 + j) * LDT + c0 + jj], x[j], x[jj]);
            pin16(x);
        }
#pragma unroll
        for (int j = 0; j < 16; ++j)
            X[lane * LDT + c0 + j] = x[j];
    }
    __builtin_amdgcn_wave_barrier();
    lds_fence_compiler();
    /* the panel's rank-16 term on the rest of the tile (blocks of 16 x 16) */
    for (int a = q + 1; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int r0 = UPPER ? 16 * a : 16 * b, cb = UPPER ? 16 * b : 16 * a;
            V acc;
            acc_load<double>(acc, X + r0 * LDT + cb, LDT);
            if (UPPER) /* U rows r0..: -= L(S)[r0.., c0..] * U12[c0.., cb..] */
                wave_mma16<double, 16>(
                    acc, [&](int r, int k) { return -S[(r0 + r) * LDT + c0 + k]; },
                    [&](int k, int c) { return X[(c0 + k) * LDT + cb + c]; });
            else /* L columns cb..: -= L21[r0.., c0..] * U(S)[c0.., cb..] */
                wave_mma16<double, 16>(
                    acc, [&](int r, int k) { return -X[(r0 + r) * LDT + c0 + k]; },
                    [&](int k, int c) { return S[(c0 + k) * LDT + cb + c]; });
            acc_store<double>(acc, X + r0 * LDT + cb, LDT);
        }
}

/*
 * Band Doolittle LU by one workgroup.  With kl, ku <= 64 the matrix is block
 * tridiagonal in 64 x 64 tiles and, without pivoting, so are its factors:
 * block step k factors the diagonal tile S_k (Eq. 6-a), turns the tile to its
 * right into U_{k,k+1} = L_kk^{-1} A_{k,k+1} and the one below it into
 * L_{k+1,k} = A_{k+1,k} U_kk^{-1}, and takes the next diagonal tile
 * S_{k+1} = A_{k+1,k+1} - L_{k+1,k} U_{k,k+1} (Eq. 6-c) on the matrix cores.
 * The two off-diagonal tiles are solved a 16-wide panel at a time by waves 1
 * and 2 while wave 0 factors the next panel of S_k (band_panel, in
 * tile_lu16's hook), so after the factorization only the last panel's pieces
 * and the product remain.  All three tiles stay in LDS; the band tiles of the
 * next step are requested a step ahead and parked after the product.
 * Entries outside the band stay exactly zero and are never stored.
 */
__global__ __launch_bounds__(NT) void k_band_factor(double *AB, int64_t ldab, int n, int kl, int ku, int32_t *info)
{
    __shared__ BandSmem sm;
    const int nt = (n + TB - 1) / TB;
    const int c = launder((int)threadIdx.x & 63), r0 = launder((int)threadIdx.x >> 6);
    const int w = wave_id(), lane = threadIdx.x & 63, lr = lane & 15, lk = lane >> 4;
    const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
    auto tile = [&](int rb, int cb) { return BandTile(AB, ldab, n, kl, ku, rb, cb); };
    /* element (r, c) of the accumulator layout */
    auto arow = [&](int bi, int r) { return wm + 16 * bi + acc_row<double>(launder(lk), r); };
    auto acol = [&](int bj) { return wn + 16 * bj + launder(lr); };
    /* the tiles right of and below S_k, unmasked, a step ahead (tile_xfer's
     * element order); parked masked */
    double a12[16], a21[16];
    auto fetch_side = [&](int kb) {
        const BandTile tu = tile(kb, kb + 1), tl = tile(kb + 1, kb);
        const int rr = launder(r0), cc = launder(c);
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            a12[i] = tu.raw(rr + 4 * i, cc);
            a21[i] = tl.raw(rr + 4 * i, cc);
        }
    };
    auto park_side = [&](int kb) {
        const BandTile tu = tile(kb, kb + 1), tl = tile(kb + 1, kb);
        const int rr = launder(r0), cc = launder(c);
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            sm.u[(rr + 4 * i) * LDT + cc] = tu.in(rr + 4 * i, cc) ? a12[i] : 0.0;
            sm.l[(rr + 4 * i) * LDT + cc] = tl.in(rr + 4 * i, cc) ? a21[i] : 0.0;
        }
    };
    int zero_at = 0;
    {
        const BandTile t0 = tile(0, 0);
        tile_xfer<double>(
            [&](int r, int cc) {
                const double v = t0.raw(r, cc);
                return t0.in(r, cc) ? v : (r == cc ? 1.0 : 0.0); /* the identity past the end */
            },
            [&](int r, int cc, double v) { sm.s[r * LDT + cc] = v; });
        if (nt > 1) {
            fetch_side(0);
            park_side(0);
        }
    }
    __syncthreads();
#pragma unroll 1
    for (int kb = 0; kb < nt; ++kb) {
        const bool last = kb + 1 == nt, more = kb + 2 < nt;
        const BandTile td = tile(kb, kb), tu = tile(kb, kb + 1), tl = tile(kb + 1, kb), tn = tile(kb + 1, kb + 1);
        Acc64<double> acc;
        if (!last) {
#pragma unroll
            for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                for (int bj = 0; bj < 2; ++bj)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        acc.v[bi][bj][r] = tn.raw(arow(bi, r), acol(bj));
        }
        if (more)
            fetch_side(kb + 1);
        const int z = tile_lu16(sm.s, sm.rinv, sm.aux, min(TB, n - kb * TB), &sm.zflag,
                                [&](int q, int stage) __attribute__((always_inline)) {
                                    if (last || stage != 0)
                                        return;
                                    if (wave_id() == 1)
                                        band_panel<true>(sm.s, sm.rinv, sm.u, q);
                                    else if (wave_id() == 2)
                                        band_panel<false>(sm.s, sm.rinv, sm.l, q);
                                });
        if (z && !zero_at)
            zero_at = kb * TB + z;
        tile_xfer<double>([&](int r, int cc) { return sm.s[r * LDT + cc]; },
                          [&](int r, int cc, double v) {
                              if (td.in(r, cc))
                                  *td.addr(r, cc) = v;
                          });
        if (last)
            break;
        /* the last panel's pieces */
        if (w == 1)
            band_panel<true>(sm.s, sm.rinv, sm.u, 3);
        else if (w == 2)
            band_panel<false>(sm.s, sm.rinv, sm.l, 3);
        __syncthreads();
        tile_xfer<double>([&](int r, int cc) { return sm.u[r * LDT + cc]; },
                          [&](int r, int cc, double v) {
                              if (tu.in(r, cc))
                                  *tu.addr(r, cc) = v;
                          });
        tile_xfer<double>([&](int r, int cc) { return sm.l[r * LDT + cc]; },
                          [&](int r, int cc, double v) {
                              if (tl.in(r, cc))
                                  *tl.addr(r, cc) = v;
                          });
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int rr = arow(bi, r), cc = acol(bj);
                    acc.v[bi][bj][r] = tn.in(rr, cc) ? acc.v[bi][bj][r] : (rr == cc ? 1.0 : 0.0);
                }
        /* L_{k+1,k} (upper) times U_{k,k+1} (lower): inner indices
         * k >= max(r, c), for the wave's quadrant from max(wm, wn) */
        acc64_mma_range<double, true>(acc, [&](int r, int k) { return sm.l[r * LDT + k]; },
                                      [&](int k, int cc) { return sm.u[k * LDT + cc]; }, max(wm, wn), TB);
        acc64_store(acc, LdsTile<double>{sm.s});
        __syncthreads();
        if (more) {
            park_side(kb + 1);
            __syncthreads();
        }
    }
    if (threadIdx.x == 0 && info)
        *info = zero_at;
}

/*
 * Operands of the band substitutions, one workgroup per 64-row block b (all
 * independent), four 64 x 64 tiles (pitch 64) at P + b * 4 * 4096: L_bb^{-1}
 * (unit diagonal and zeros above written out), U_bb^{-1} (zeros below), the
 * band tile L_{b,b-1} left of the diagonal and the band tile U_{b,b+1} right
 * of it (zero where the band or the matrix has no element).  The inverses
 * come from the factored diagonal tile (tile_inv16; a partial last tile is
 * padded with the identity).  With every mask applied here, the sweep reads
 * contiguous, unmasked operands.
 */
constexpr int kBandSolveTiles = 4;

__global__ __launch_bounds__(NT) void k_band_packs(const double *AB, int64_t ldab, int n, int kl, int ku,
                                                   double *__restrict__ P)
{
    __shared__ TileSmem<double> sm;
    const int b = blockIdx.x, nt = (n + TB - 1) / TB;
    double *AB_ = const_cast<double *>(AB);
    const BandTile t(AB_, ldab, n, kl, ku, b, b);
    tile_xfer<double>(
        [&](int r, int c) {
            const double v = t.raw(r, c);
            return t.in(r, c) ? v : (r == c ? 1.0 : 0.0);
        },
        [&](int r, int c, double v) { sm.t0[r * LDT + c] = v; });
    __syncthreads();
    if (threadIdx.x < TB)
        sm.rinv[threadIdx.x] = recip(sm.t0[threadIdx.x * LDT + threadIdx.x]);
    __syncthreads();
    tile_inv16(sm.t0, sm.rinv, sm.t1);
    double *Pb = P + (int64_t)b * kBandSolveTiles * TB * TB;
    tile_xfer<double>(
        [&](int r, int c) { return sm.t1[r * LDT + c]; },
        [&](int r, int c, double v) {
            Pb[r * TB + c] = r > c ? v : (r == c ? 1.0 : 0.0);
            Pb[TB * TB + r * TB + c] = r <= c ? v : 0.0;
        });
    /* the off-diagonal band tiles (the first block's left one and the last
     * block's right one lie outside the matrix: zero) */
    const BandTile tlft(AB_, ldab, n, kl, ku, b, b - 1), trgt(AB_, ldab, n, kl, ku, b, b + 1);
    const bool has_l = b > 0, has_r = b + 1 < nt;
    tile_xfer<double>(
        [&](int r, int c) {
            const double v = tlft.raw(r, c);
            return (has_l && tlft.in(r, c)) ? v : 0.0;
        },
        [&](int r, int c, double v) { Pb[2 * TB * TB + r * TB + c] = v; });
    tile_xfer<double>(
        [&](int r, int c) {
            const double v = trgt.raw(r, c);
            return (has_r && trgt.in(r, c)) ? v : 0.0;
        },
        [&](int r, int c, double v) { Pb[3 * TB * TB + r * TB + c] = v; });
}

/*
 * Band substitutions (Eq. 7) by one workgroup for up to 16 right-hand sides,
 * 64-row blocks in order:
 *   forward,  y_b = L_bb^{-1} (b_b - L_{b,b-1} y_{b-1}),
 *   backward, x_b = U_bb^{-1} (y_b - U_{b,b+1} x_{b+1}).
 * Each block is two 64 x 64 by 64 x 16 products on the matrix cores (wave w
 * the rows 16w..16w+15; lane group g supplies inner indices 16q + 4g .. +3,
 * contiguous in the operand tiles of k_band_packs, so a lane loads each
 * group of four as one 32-byte vector), the operands of a block loaded two
 * blocks ahead in a ring of three register sets.  The previous block's
 * solution stays in LDS for the next product; each solved block is written
 * to B.
 */
constexpr int BXP = 17; /* LDS pitch of a 64 x 16 block of right-hand sides */

struct BandSweepOps {
    d4 a1[4], a2[4]; /* off-diagonal band tile, diagonal tile's inverse */
    double y[4];     /* the block's right-hand sides (accumulator layout) */
};

struct BandSweepArgs {
    int n;
    const double *P;
    double *B;
    int64_t ldb;
    int nrhs_here;
};

template <bool FWD>
__device__ __forceinline__ void band_sweep_load(const BandSweepArgs &a, int b, BandSweepOps &o)
{
    const int w = wave_id(), lane = threadIdx.x & 63, lr = lane & 15, lk = lane >> 4;
    const int row = 16 * w + lr, b0 = b * TB;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int rb = b0 + 16 * w + acc_row<double>(lk, r);
        o.y[r] = a.B[(rb < a.n && lr < a.nrhs_here) ? (int64_t)rb * a.ldb + lr : 0];
    }
    const double *Pb = a.P + (int64_t)b * kBandSolveTiles * TB * TB + row * TB + 4 * lk;
    const double *Pinv = Pb + (FWD ? 0 : TB * TB), *Poff = Pb + (FWD ? 2 : 3) * TB * TB;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        o.a1[q] = *reinterpret_cast<const d4 *>(Poff + 16 * q);
        o.a2[q] = *reinterpret_cast<const d4 *>(Pinv + 16 * q);
    }
}

template <bool FWD>
__device__ __forceinline__ void band_sweep_block(const BandSweepArgs &a, const BandSweepOps &o, bool has_off, int b,
                                                 double *xs, double *ys)
{
    const int w = wave_id(), lane = threadIdx.x & 63, lr = lane & 15, lk = lane >> 4;
    const int b0 = b * TB;
    d4 acc;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int rb = b0 + 16 * w + acc_row<double>(lk, r);
        acc[r] = (rb < a.n && lr < a.nrhs_here) ? o.y[r] : 0.0;
    }
    if (has_off)
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int ks = 0; ks < 4; ++ks)
                acc = mfma16(-o.a1[q][ks], xs[(16 * q + 4 * lk + ks) * BXP + lr], acc);
#pragma unroll
    for (int r = 0; r < 4; ++r)
        ys[(16 * w + acc_row<double>(lk, r)) * BXP + lr] = acc[r];
    __syncthreads();
    d4 x = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int ks = 0; ks < 4; ++ks)
            x = mfma16(o.a2[q][ks], ys[(16 * q + 4 * lk + ks) * BXP + lr], x);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int rr = 16 * w + acc_row<double>(lk, r), rb = b0 + rr;
        xs[rr * BXP + lr] = x[r];
        if (rb < a.n && lr < a.nrhs_here)
            a.B[(int64_t)rb * a.ldb + lr] = x[r];
    }
    __syncthreads();
}

template <bool FWD> __device__ __forceinline__ void band_sweep(const BandSweepArgs &a, double *xs, double *ys)
{
    const int nt = (a.n + TB - 1) / TB;
    auto blk = [&](int i) { return FWD ? i : nt - 1 - i; };
    /* three operand sets in a ring: each block's loads are issued two
     * blocks before it is solved */
    BandSweepOps o[3];
    band_sweep_load<FWD>(a, blk(0), o[0]);
    if (nt > 1)
        band_sweep_load<FWD>(a, blk(1), o[1]);
#pragma unroll 1
    for (int i = 0; i < nt; i += 3) {
        if (i + 2 < nt)
            band_sweep_load<FWD>(a, blk(i + 2), o[2]);
        band_sweep_block<FWD>(a, o[0], i > 0, blk(i), xs, ys);
        if (i + 1 >= nt)
            break;
        if (i + 3 < nt)
            band_sweep_load<FWD>(a, blk(i + 3), o[0]);
        band_sweep_block<FWD>(a, o[1], true, blk(i + 1), xs, ys);
        if (i + 2 >= nt)
            break;
        if (i + 4 < nt)
            band_sweep_load<FWD>(a, blk(i + 4), o[1]);
        band_sweep_block<FWD>(a, o[2], true, blk(i + 2), xs, ys);
    }
}

__global__ __launch_bounds__(NT) void k_band_solve(BandSweepArgs a)
{
    __shared__ double xs[TB * BXP], ys[TB * BXP];
    band_sweep<true>(a, xs, ys);
    band_sweep<false>(a, xs, ys);
}

hipError_t band_factor(double *AB, int64_t ldab, int n, int kl, int ku, int32_t *info, hipStream_t st)
{
    hipLaunchKernelGGL(k_band_factor, dim3(1), dim3(NT), 0, st, AB, ldab, n, kl, ku, info);
    return hipGetLastError();
}

hipError_t band_solve(const double *AB, int64_t ldab, int n, int kl, int ku, double *B, int64_t ldb, int nrhs,
                      double *P, hipStream_t st)
{
    const int nt = (n + TB - 1) / TB;
    hipLaunchKernelGGL(k_band_packs, dim3(nt), dim3(NT), 0, st, AB, ldab, n, kl, ku, P);
    hipError_t e = hipGetLastError();
    for (int c0 = 0; c0 < nrhs && e == hipSuccess; c0 += 16) {
        const BandSweepArgs a{n, P, B + c0, ldb, min(16, nrhs - c0)};
        hipLaunchKernelGGL(k_band_solve, dim3(1), dim3(NT), 0, st, a);
        e = hipGetLastError();
    }
    return e;
}

/* ---------------------------------------------------- explicit inverse --- */

/* Inverse packs of every 64 x 64 diagonal tile of a factored system (one
 * workgroup per tile, all independent): tile_inv16 of the factored tile,
 * stored 64 x 64 (pitch 64) at P + b * 4096 -- the inverse of its unit lower
 * factor in the strict lower part, the inverse of its upper factor in the
 * upper part. */
template <typename T>
__global__ __launch_bounds__(NT) void k_diag_packs(const T *__restrict__ LU, int64_t lda, int n, T *__restrict__ P)
{
    __shared__ TileSmem<T> sm;
    const int b = blockIdx.x, k0 = b * TB, kw = min(TB, n - k0);
    stage_tile_identity(sm.t0, LU + (int64_t)k0 * lda + k0, lda, kw, kw);
    __syncthreads();
    if (threadIdx.x < TB)
        sm.rinv[threadIdx.x] = recip(sm.t0[threadIdx.x * LDT + threadIdx.x]);
    __syncthreads();
    tile_inv16(sm.t0, sm.rinv, sm.t1);
    T *Pb = P + (int64_t)b * TB * TB;
    tile_xfer<T>([&](int r, int c) { return sm.t1[r * LDT + c]; }, [&](int r, int c, T v) { Pb[r * TB + c] = v; });
}

/*
 * Explicit inverse X = A^{-1} = U^{-1} L^{-1} from the factors (Eq. 4-c: the
 * elementary upper factors times the elementary lower factors), as two
 * right-looking blocked triangular solves on the identity, one launch per
 * 64-wide block step, one workgroup per 64 x 64 tile of the result:
 *   forward, W = L^{-1} (block lower triangular): step k takes the tiles
 *     (r, c), r > k, c <= k, and subtracts L_rk W_kc (a tile first touched
 *     here starts from zero); the workgroup of block row k + 1 then has its
 *     last update and applies L_{k+1,k+1}^{-1} at once; one more workgroup
 *     writes the diagonal tile W_{k+1,k+1} = L_{k+1,k+1}^{-1};
 *   backward, X = U^{-1} W (dense): the tiles of row r < k take the terms
 *     U_rs X_sc of the steps s >= k G = kInvGroup steps at a time: launch
 *     k updates the rows r = k-1, k-1-G, ... with the terms of steps k ..
 *     k+G-1 (one stream with K = 64 G over contiguous columns of U and rows
 *     of X; fewer at the first such launch), so a tile is read and written
 *     once per G steps; the tiles above W's diagonal start from zero at
 *     their first update; block row k - 1 has then received every term and
 *     applies U_{k-1,k-1}^{-1}.
 * W is kept in X's storage and overwritten in place.  The inverses of the
 * diagonal tiles come from their packs (k_diag_packs).
 */
constexpr int kInvGroup = 2; /* backward steps applied per tile update */

template <typename T, bool FWD>
__global__ __launch_bounds__(NT, 2) void k_inv_step(const T *__restrict__ LU, int64_t lda, int n,
                                                    const T *__restrict__ P, T *__restrict__ X, int64_t ldx, int k)
{
    __shared__ TileSmem<T> sm;
    const int nt = (n + TB - 1) / TB, b = blockIdx.x;
    int r, c;
    bool diag_only = false;
    if (FWD) {
        const int cols = k + 1, nupd = (nt - 1 - k) * cols;
        if (b < nupd) {
            r = k + 1 + b / cols;
            c = b % cols;
        } else {
            r = c = k + 1; /* W_{k+1,k+1} = L_{k+1,k+1}^{-1} */
            diag_only = true;
        }
    } else {
        if (k == nt) { /* the last block row: only its inverse product */
            r = nt - 1;
            c = b;
            diag_only = true;
        } else { /* rows k-1, k-1-G, ...: the terms of steps k .. k+G-1 */
            r = k - 1 - kInvGroup * (b / nt);
            c = b % nt;
        }
    }
    const int next = FWD ? k + 1 : k - 1;
    const int nr = min(TB, n - r * TB), nc = min(TB, n - c * TB);
    T *C = X + (int64_t)r * TB * ldx + (int64_t)c * TB;
    const T *Pr = P + (int64_t)r * TB * TB;
    if (FWD && diag_only) {
        tile_xfer<T>(
            [&](int rr, int cc) {
                const T v = Pr[rr * TB + cc];
                return rr > cc ? v : (rr == cc ? T(1) : T(0));
            },
            [&](int rr, int cc, T v) {
                if (rr < nr && cc < nc)
                    C[(int64_t)rr * ldx + cc] = v;
            });
        return;
    }
    Acc64<T> acc;
    /* the running value: zero where the tile is first touched (forward: the
     * column being eliminated; backward: above W's diagonal, at the row's
     * first update, launch nt - 1 or nt - 2) */
    const bool fresh = FWD ? c == k : (r < c && k + kInvGroup >= nt);
    if (fresh)
        acc64_zero(acc);
    else
        acc64_load(acc, DenseC<T>{C, ldx, nr, nc});
    if (!diag_only) {
        /* backward: steps k .. k + G - 1, those that exist */
        const int kw = min(FWD ? TB : kInvGroup * TB, n - k * TB);
        acc64_stream<T, true>(acc, LU + (int64_t)r * TB * lda + (int64_t)k * TB, lda,
                              X + (int64_t)k * TB * ldx + (int64_t)c * TB, ldx, nr, nc, kw);
    }
    if (r != next) {
        acc64_store(acc, DenseC<T>{C, ldx, nr, nc});
        return;
    }
    /* block row `next` is complete: times its diagonal tile's inverse */
    acc64_store(acc, LdsTile<T>{sm.t0});
    tile_xfer<T>([&](int rr, int cc) { return Pr[rr * TB + cc]; },
                 [&](int rr, int cc, T v) { sm.t1[rr * LDT + cc] = v; });
    __syncthreads();
    if (FWD)
        wg_gemm64f<T, true>(DenseC<T>{C, ldx, nr, nc}, InvL<T>{sm.t1},
                            [&](int kk, int cc) { return sm.t0[kk * LDT + cc]; });
    else
        wg_gemm64f<T, true>(DenseC<T>{C, ldx, nr, nc}, InvUFull<T>{sm.t1},
                            [&](int kk, int cc) { return sm.t0[kk * LDT + cc]; });
}

template <typename T>
hipError_t lu_inverse(const T *LU, int64_t lda, int n, T *X, int64_t ldx, T *P, hipStream_t st)
{
    const int nt = (n + TB - 1) / TB;
    hipLaunchKernelGGL(k_diag_packs<T>, dim3(nt), dim3(NT), 0, st, LU, lda, n, P);
    hipError_t e = hipGetLastError();
    for (int k = -1; k + 1 < nt && e == hipSuccess; ++k) {
        const int grid = (nt - 1 - k) * (k + 1) + 1;
        hipLaunchKernelGGL((k_inv_step<T, true>), dim3(grid), dim3(NT), 0, st, LU, lda, n, (const T *)P, X, ldx, k);
        e = hipGetLastError();
    }
    for (int k = nt; k > 0 && e == hipSuccess; --k) {
        const int grid = k == nt ? nt : (k + kInvGroup - 1) / kInvGroup * nt; /* rows k-1, k-1-G, ... */
        hipLaunchKernelGGL((k_inv_step<T, false>), dim3(grid), dim3(NT), 0, st, LU, lda, n, (const T *)P, X, ldx, k);
        e = hipGetLastError();
    }
    return e;
}

/* ------------------------------------------------------- skyline (profile) --- */

/* Tile (I, J) of the block envelope (nullptr outside it). */
__device__ __forceinline__ double *sky_tile(const SkyPlan &pl, double *tiles, int I, int J)
{
    if (J <= I)
        return J >= pl.F[I] ? tiles + (int64_t)(pl.LTo[I] + J - pl.F[I]) * TB * TB : nullptr;
    return I >= pl.G[J] ? tiles + (int64_t)(pl.LTo[pl.nt] + pl.UTo[J] + I - pl.G[J]) * TB * TB : nullptr;
}

/* Pack (or unpack) the skyline arrays and the envelope tiles: workgroup b < nt
 * takes the lower tiles of block row b (lanes over columns: a row of L is
 * contiguous), b >= nt the upper tiles of block column b - nt (lanes over
 * rows: a column of U is contiguous).  Elements outside the element envelope
 * or past n are zero in the tiles and never written back. */
__global__ __launch_bounds__(NT) void k_sky_pack(SkyPlan pl, const int32_t *__restrict__ f,
                                                 const int64_t *__restrict__ rp, double *__restrict__ AL,
                                                 const int32_t *__restrict__ g, const int64_t *__restrict__ cp,
                                                 double *__restrict__ AU, double *__restrict__ tiles, int unpack)
{
    const int b = blockIdx.x, n = pl.n, lane = threadIdx.x & 63, r4 = threadIdx.x >> 6;
    const bool lower = b < pl.nt;
    const int I0 = lower ? b : pl.G[b - pl.nt], I1 = lower ? b : b - pl.nt - 1;
    const int J0 = lower ? pl.F[b] : b - pl.nt, J1 = lower ? b : b - pl.nt;
    for (int I = I0; I <= I1; ++I)
        for (int J = J0; J <= J1; ++J) {
            double *T = sky_tile(pl, tiles, I, J);
            for (int k = r4; k < TB; k += 4) {
                /* lower tiles: row r = k, column c = lane; upper: column c = k, row r = lane */
                const int r = lower ? k : lane, c = lower ? lane : k;
                const int i = I * TB + r, j = J * TB + c;
                double *p = nullptr;
                if (i < n && j < n) {
                    if (j < i)
                        p = j >= f[i] ? AL + rp[i] + (j - f[i]) : nullptr;
                    else
                        p = i >= g[j] ? AU + cp[j] + (i - g[j]) : nullptr;
                }
                if (unpack) {
                    if (p)
                        *p = T[r * TB + c];
                } else {
                    T[r * TB + c] = p ? *p : 0.0;
                }
            }
        }
}

/*
 * Skyline LU on the envelope tiles, right-looking (Eq. 6-a/6-c restricted to
 * the envelope, which the elimination keeps: if L_IJ and U_JK exist, so does
 * tile (I, K)), one launch per block step J whose workgroups take their roles
 * from a ticket (the first to arrive is the diagonal one, so the waits below
 * always end):
 *   role 0, the diagonal tile: receives step J-1's rank-64 term, is factored
 *     (tile_lu16), and the inverses of its factors are published (P, then a
 *     flag) for the panel tiles;
 *   the panel tiles (I, J) below and (J, I) right of it in the envelope:
 *     each receives step J-1's term, waits for the flag, and is multiplied by
 *     the diagonal tile's inverses;
 *   the other tiles (I, K), I, K > J, for which L_{I,J-1} and U_{J-1,K}
 *     exist: each receives step J-1's term, all in parallel.
 * A tile has thereby received the terms of all the steps before its own when
 * it is factored or solved, and the long inner products of the block Crout
 * order are spread over the launches as rank-64 terms off the chain.  Tiles
 * outside the envelope stay zero and are never touched.  ctl: the status word
 * (bounded waits), then per step a ticket counter and the flag.
 */
__device__ __forceinline__ int sky_nth(const int16_t *X, int from, int nt, int lim, int cnt)
{
    /* the cnt-th block index x >= from with X[x] <= lim, or -1: 64 entries
     * per round, one per lane (a scan entry by entry waits for each load),
     * the hit picked from the wave's ballot; every wave gets the same */
    const int lane = threadIdx.x & 63;
    for (int base = from; base < nt; base += 64) {
        const int x = base + lane;
        const int16_t v = X[min(x, nt - 1)];
        const unsigned long long m = __ballot(x < nt && v <= lim);
        const int c = __popcll(m);
        if (cnt < c) {
            unsigned long long mm = m;
            for (int i = 0; i < cnt; ++i)
                mm &= mm - 1;
            return base + __ffsll((long long)mm) - 1;
        }
        cnt -= c;
    }
    return -1;
}

__global__ __launch_bounds__(NT) void k_sky_step(SkyPlan pl, double *__restrict__ tiles, double *__restrict__ P,
                                                 int J, int nl, int nu, int nlp, int nup, int *ctl, int32_t *info,
                                                 long wlim)
{
    __shared__ TileSmem<double> sm;
    __shared__ int s_ticket;
    const int n = pl.n, nt = pl.nt;
    int *status = ctl, *ticket = ctl + kCtlHead + 2 * J, *flag = ticket + 1;
    if (threadIdx.x == 0) {
        s_ticket = atomicAdd(ticket, 1);
        sm.avail = 0;
    }
    __syncthreads();
    int q = s_ticket;
    const int kJ = min(TB, n - J * TB);
    /* step J-1's rank-64 term for tile (I, K): L_{I,J-1} U_{J-1,K}, when both exist */
    auto pending = [&](Acc64<double> &acc, int I, int K, int nr, int nc) {
        if (J == 0 || pl.F[I] > J - 1 || pl.G[K] > J - 1)
            return;
        acc64_stream_pairs(
            acc, 1,
            [&](int, const double *&a, const double *&b) {
                a = sky_tile(pl, tiles, I, J - 1);
                b = sky_tile(pl, tiles, J - 1, K);
            },
            nr, nc);
    };
    double *D = sky_tile(pl, tiles, J, J);
    if (q == 0) { /* the diagonal tile */
        Acc64<double> acc;
        acc64_load(acc, DenseC<double>{D, TB, kJ, kJ});
        pending(acc, J, J, kJ, kJ);
        acc64_store(acc, LdsTile<double>{sm.t0});
        __syncthreads();
        if (threadIdx.x >= kJ && threadIdx.x < TB)
            sm.t0[threadIdx.x * LDT + threadIdx.x] = 1.0;
        __syncthreads();
        const bool pub = nl + nu > 0;
        /* what the panel tiles read, published 16 columns at a time: for
         * panel p of the factored tile, roles 0 and 1 the inverses of its
         * diagonal block's factors (to P), role 2 the block itself and its L
         * part below and U part to the right (to D, the parts the panel
         * tiles read device-coherent); stage 0 issues the stores, stage 1
         * waits for them and counts them in the flag (3 per panel) */
        auto publish_panel = [&](int p, int role, int stage) __attribute__((always_inline)) {
            const int l = threadIdx.x & 63, b0 = 16 * p;
            if (stage == 1) {
                if (role <= 2) {
                    __builtin_amdgcn_s_waitcnt(0);
                    if (l == 0)
                        __hip_atomic_fetch_add(flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                return;
            }
            auto put = [&](int i, int c, double v) __attribute__((always_inline)) {
                store_coherent(P + (b0 + i) * TB + b0 + c, v);
            };
            if (role == 0) {
                diag_block_inv<double, false>(sm.t0, sm.rinv, p, put);
            } else if (role == 1) {
                diag_block_inv<double, true>(sm.t0, sm.rinv, p, put);
            } else if (role == 2) {
                for (int idx = l; idx < 256; idx += 64) {
                    const int r = b0 + (idx >> 4), c = b0 + (idx & 15);
                    if (r < kJ && c < kJ)
                        D[r * TB + c] = sm.t0[r * LDT + c];
                }
                for (int idx = l; idx < (48 - b0) * 16; idx += 64) {
                    const int a = b0 + 16 + (idx >> 4), c = b0 + (idx & 15);
                    if (a < kJ && c < kJ) {
                        store_coherent(D + a * TB + c, sm.t0[a * LDT + c]);
                        store_coherent(D + c * TB + a, sm.t0[c * LDT + a]);
                    }
                }
            }
        };
        /* panels 0..2 are published by waves 1..3 while wave 0 factors the
         * next panel; the last one after the factorization */
        const int z = tile_lu16(sm.t0, sm.rinv, sm.aux, kJ, &sm.zflag, [&](int p, int stage) __attribute__((always_inline)) {
            if (pub)
                publish_panel(p, wave_id() - 1, stage);
        });
        if (threadIdx.x == 0 && info && (J == 0 || (z && *info == 0)))
            *info = z ? J * TB + z : 0;
        if (pub) {
            if (wave_id() >= 1) /* panel 2's stores, issued while panel 3 was factored */
                publish_panel(2, wave_id() - 1, 1);
            publish_panel(3, wave_id(), 0);
            publish_panel(3, wave_id(), 1);
        } else {
            lds_store_tile(sm.t0, D, TB, kJ, kJ);
        }
        return;
    }
    q -= 1;
    if (q < nl + nu) { /* a panel tile */
        const bool lower = q < nl;
        const int I = lower ? sky_nth(pl.F, J + 1, nt, J, q) : sky_nth(pl.G, J + 1, nt, J, q - nl);
        if (I < 0)
            return;
        const int kI = min(TB, n - I * TB);
        const int r0 = lower ? I : J, c0 = lower ? J : I, nr = lower ? kI : kJ, nc = lower ? kJ : kI;
        double *G = sky_tile(pl, tiles, r0, c0);
        Acc64<double> acc;
        acc64_load(acc, DenseC<double>{G, TB, nr, nc});
        pending(acc, r0, c0, nr, nc);
        acc64_store(acc, LdsTile<double>{sm.t0});
        __syncthreads();
        /* the solve against the factored diagonal tile, block step p as soon
         * as strip p is published (the flag counts 3 per strip): each wave
         * keeps its 16-wide slab of the tile in accumulators (transposed for
         * the L tiles, L_IJ = A_IJ U_JJ^{-1} solved as U^T X^T = A^T) and runs
         * step p with the strip staged in t1: the diagonal block times the
         * inverse of the strip's diagonal block, then its contribution
         * removed from the blocks after it, each product taking the finished
         * block as its B operand */
        const bool from_right = lower; /* L_IJ = A_IJ U_JJ^{-1}: U^{-1} applied from the right */
        const int w = wave_id(), l = threadIdx.x & 63, lr = l & 15, lk = l >> 4;
        d4 a[4];
#pragma unroll
        for (int q2 = 0; q2 < 4; ++q2)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                a[q2][r] = from_right ? sm.t0[(16 * w + lr) * LDT + 16 * q2 + acc_row<double>(lk, r)]
                                 : sm.t0[(16 * q2 + acc_row<double>(lk, r)) * LDT + 16 * w + lr];
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            wait_solved(flag, 3 * p + 2, &sm.avail, status, wlim);
            /* strip p: for a U tile rows 16p.. of columns 16p..16p+15 (L),
             * for an L tile columns 16p.. of rows 16p..16p+15 (U); diagonal
             * block from P, identity past the matrix end */
            const int len = 64 - 16 * p;
            double v[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int idx = threadIdx.x + NT * i;
                const int r = from_right ? 16 * p + idx / len : 16 * p + (idx >> 4);
                const int c = from_right ? 16 * p + idx % len : 16 * p + (idx & 15);
                v[i] = idx >= len * 16           ? 0.0
                       : (r >> 4) == (c >> 4)    ? load_coherent(P + r * TB + c)
                       : (r < kJ && c < kJ)      ? load_coherent(D + r * TB + c)
                                                 : 0.0;
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int idx = threadIdx.x + NT * i;
                const int r = from_right ? 16 * p + idx / len : 16 * p + (idx >> 4);
                const int c = from_right ? 16 * p + idx % len : 16 * p + (idx & 15);
                if (idx < len * 16)
                    sm.t1[r * LDT + c] = v[i];
            }
            __syncthreads();
            d4 x = {0.0, 0.0, 0.0, 0.0};
            if (from_right) {
                wave_mma16_acc<double>(
                    x,
                    [&](int r, int k) {
                        const double u = sm.t1[(16 * p + k) * LDT + 16 * p + r];
                        return k <= r ? u : 0.0;
                    },
                    a[p]);
                a[p] = x;
#pragma unroll
                for (int q2 = p + 1; q2 < 4; ++q2)
                    wave_mma16_acc<double>(a[q2], [&](int r, int k) { return -sm.t1[(16 * p + k) * LDT + 16 * q2 + r]; },
                                           a[p]);
            } else {
                wave_mma16_acc<double>(
                    x,
                    [&](int r, int k) {
                        const double u = sm.t1[(16 * p + r) * LDT + 16 * p + k];
                        return r > k ? u : (r == k ? 1.0 : 0.0);
                    },
                    a[p]);
                a[p] = x;
#pragma unroll
                for (int q2 = p + 1; q2 < 4; ++q2)
                    wave_mma16_acc<double>(a[q2], [&](int r, int k) { return -sm.t1[(16 * q2 + r) * LDT + 16 * p + k]; },
                                           a[p]);
            }
        }
        __syncthreads();
#pragma unroll
        for (int q2 = 0; q2 < 4; ++q2)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                if (from_right)
                    sm.t0[(16 * w + lr) * LDT + 16 * q2 + acc_row<double>(lk, r)] = a[q2][r];
                else
                    sm.t0[(16 * q2 + acc_row<double>(lk, r)) * LDT + 16 * w + lr] = a[q2][r];
            }
        __syncthreads();
        lds_store_tile(sm.t0, G, TB, nr, nc);
        return;
    }
    q -= nl + nu;
    if (q >= nlp * nup)
        return;
    { /* a trailing tile (I, K), I, K > J: step J-1's term only */
        const int I = sky_nth(pl.F, J + 1, nt, J - 1, q / nup), K = sky_nth(pl.G, J + 1, nt, J - 1, q % nup);
        if (I < 0 || K < 0)
            return;
        const int nr = min(TB, n - I * TB), nc = min(TB, n - K * TB);
        double *C = sky_tile(pl, tiles, I, K);
        Acc64<double> acc;
        acc64_load(acc, DenseC<double>{C, TB, nr, nc});
        pending(acc, I, K, nr, nc);
        acc64_store(acc, DenseC<double>{C, TB, nr, nc});
    }
}

hipError_t skyline_factor(const SkyPlan &pl, double *tiles, double *P, int *ctl, int32_t *info, long wlim,
                          hipStream_t st)
{
    hipError_t e = fill_i32(ctl, kCtlHead + 2 * pl.nt, 0, st);
    for (int J = 0; J < pl.nt && e == hipSuccess; ++J) {
        int nl = 0, nu = 0, nlp = 0, nup = 0;
        for (int I = J + 1; I < pl.nt; ++I) {
            nl += pl.F[I] <= J;
            nu += pl.G[I] <= J;
            nlp += pl.F[I] <= J - 1;
            nup += pl.G[I] <= J - 1;
        }
        const int grid = 1 + nl + nu + nlp * nup;
        hipLaunchKernelGGL(k_sky_step, dim3(grid), dim3(NT), 0, st, pl, tiles, P, J, nl, nu, nlp, nup, ctl, info,
                           wlim);
        e = hipGetLastError();
    }
    if (e == hipSuccess && info)
        e = fold_status(ctl, info, st);
    return e;
}

/* Operator tiles of the skyline factors for solve_block (zero outside the
 * envelope). */
template <int MODE> struct SkyOp {
    const SkyPlan *pl;
    const double *tiles;
    __device__ __forceinline__ void operator()(double *S, int bi, int bj) const
    {
        const double *T = sky_tile(*pl, const_cast<double *>(tiles), bi, bj);
        const int nr = min(TB, pl->n - bi * TB), nc = min(TB, pl->n - bj * TB);
        tile_xfer<double>([&](int r, int c) { return (T && r < nr && c < nc) ? T[r * TB + c] : 0.0; },
                          [&](int r, int c, double v) { S[r * LDT + c] = v; });
    }
    /* the tile's row rr, columns 16q.., read unconditionally (clamped into
     * the tile) and masked after; a tile outside the envelope reads as zero */
    __device__ __forceinline__ void seg(int bi, int bj, int rr, int q, double (&m)[16]) const
    {
        const double *T = sky_tile(*pl, const_cast<double *>(tiles), bi, bj);
        const int nr = min(TB, pl->n - bi * TB), nc = min(TB, pl->n - bj * TB);
        if (!T) {
#pragma unroll
            for (int cc = 0; cc < 16; ++cc)
                m[cc] = 0.0;
            return;
        }
        const double *row = T + min(rr, nr - 1) * TB;
#pragma unroll
        for (int cc = 0; cc < 16; ++cc) {
            const int c = 16 * q + cc;
            const double v = row[min(c, nc - 1)];
            m[cc] = (rr < nr && c < nc) ? v : 0.0;
        }
    }
};

/* Inverse packs of the skyline factor's diagonal tiles, one workgroup per
 * tile (all independent): P + b * 4096 (pitch 64) receives L_bb^{-1} in its
 * strict lower part (unit diagonal implied) and U_bb^{-1} in its upper part;
 * a partial last tile is padded with the identity. */
__global__ __launch_bounds__(NT) void k_sky_packs(SkyPlan pl, const double *__restrict__ tiles,
                                                  double *__restrict__ P)
{
    __shared__ TileSmem<double> sm;
    const int b = blockIdx.x, kb = min(TB, pl.n - b * TB);
    stage_tile_identity(sm.t0, sky_tile(pl, const_cast<double *>(tiles), b, b), TB, kb, kb);
    __syncthreads();
    if (threadIdx.x < TB)
        sm.rinv[threadIdx.x] = recip(sm.t0[threadIdx.x * LDT + threadIdx.x]);
    __syncthreads();
    tile_inv16(sm.t0, sm.rinv, sm.t1);
    double *Pb = P + (int64_t)b * TB * TB;
    tile_xfer<double>([&](int r, int c) { return sm.t1[r * LDT + c]; },
                      [&](int r, int c, double v) { Pb[r * TB + c] = v; });
}

/* The operand values one lane contributes to a pack product (below): row
 * 16w + lr of the pack of block blk, inner indices 16q + 4lk + ks, loaded
 * raw (the triangle is selected at use). */
__device__ __forceinline__ void sky_pack_load(const double *__restrict__ Pb, double (&pv)[16])
{
    const int w = wave_id(), l = threadIdx.x & 63, lr = l & 15, lk = l >> 4, row = 16 * w + lr;
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int ks = 0; ks < 4; ++ks)
            pv[4 * q + ks] = Pb[row * TB + 16 * q + 4 * lk + ks];
}

/* Block blk of a substitution with all its updates applied, its right-hand
 * sides staged in LDS (Ys, 64 x 16, pitch 17, zero past n and nrhs_here):
 * times the inverse of the diagonal tile's unit lower (LOWER) or upper
 * factor from its pack (pv, from sky_pack_load), one matrix-core product
 * (wave w the rows 16w..16w+15), the result stored in B. */
template <bool LOWER>
__device__ __forceinline__ void sky_pack_product(const double (&pv)[16], const double *Ys, int n, double *B,
                                                 int64_t ldb, int nrhs_here, int blk)
{
    constexpr int YP = 17;
    const int b0 = blk * TB;
    const int w = wave_id(), l = threadIdx.x & 63, lr = l & 15, lk = l >> 4, row = 16 * w + lr;
    d4 x = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const int k = 16 * q + 4 * lk + ks;
            const double other = (LOWER && row == k) ? 1.0 : 0.0;
            const bool keep = LOWER ? row > k : row <= k;
            x = mfma16(keep ? pv[4 * q + ks] : other, Ys[k * YP + lr], x);
        }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int rb = b0 + 16 * w + acc_row<double>(lk, r);
        if (rb < n && lr < nrhs_here)
            B[(int64_t)rb * ldb + lr] = x[r];
    }
}

/*
 * One step of the skyline substitutions (Eq. 1), FWD: L Y = B (block order
 * 0, 1, ...), else U X = Y (block order nt-1, nt-2, ...).  Block J is solved
 * already; each workgroup takes one envelope tile of block column J -- the
 * lower tiles (R, J), R > J, forward; the upper tiles (I, J), I < J, backward
 * -- and subtracts its product with block J's solution from its block row's
 * right-hand sides (distinct rows per workgroup).  The block solved next
 * (J + 1 forward, J - 1 backward) then has all its updates: the workgroup
 * that updated it (or the extra last workgroup when block J has no tile in
 * that row) solves its diagonal triangle right away, from the updated rows
 * kept in LDS and the pack's operands loaded at the start.  J = -1 (forward)
 * or nt (backward) only solves the first block.
 */
template <int NR, bool FWD>
__global__ __launch_bounds__(NT) void k_sky_sweep(SkyPlan pl, const double *__restrict__ tiles,
                                                  const double *__restrict__ P, double *B, int64_t ldb,
                                                  int nrhs_here, int J, int ntarget)
{
    constexpr int MODE = FWD ? TRI_L : TRI_U;
    constexpr int YP = 17;
    __shared__ TileSmem<double> sm;
    const int nt = pl.nt, n = pl.n, b = blockIdx.x;
    const int t = threadIdx.x, rr = t >> 2, q = t & 3;
    const SkyOp<MODE> op{&pl, tiles};
    const int next = FWD ? J + 1 : J - 1;
    int target = -1;
    if (b < ntarget) /* forward: the b-th block row below J reaching column J; backward: rows G_J.. */
        target = FWD ? sky_nth(pl.F, J + 1, nt, J, b) : pl.G[J] + b;
    else
        target = next; /* no tile of block column J in the next block's row */
    const bool solves = target == next && next >= 0 && next < nt;
    double pv[16]; /* loaded by every workgroup (block index clamped): no branch around loads */
    sky_pack_load(P + (int64_t)min(max(next, 0), nt - 1) * TB * TB, pv);
    double *Ys = sm.t0; /* the next block's right-hand sides for its pack product */
    if (b < ntarget) {
        double *Y = sm.t1;
        const int kJ = min(TB, n - J * TB);
        for (int idx = t; idx < TB * NR; idx += NT) {
            const int r = idx / NR, c = idx % NR;
            const double v = B[(int64_t)(J * TB + min(r, kJ - 1)) * ldb + min(c, nrhs_here - 1)];
            Y[r * NR + c] = (r < kJ && c < nrhs_here) ? v : 0.0;
        }
        double m[16];
        op.seg(target, J, rr, q, m);
        const int rows = min(TB, n - target * TB);
        double bo[NR]; /* row rr's right-hand sides (address clamped) */
        {
            const double *brow = B + (int64_t)(target * TB + min(rr, rows - 1)) * ldb;
#pragma unroll
            for (int c = 0; c < NR; ++c)
                bo[c] = brow[min(c, nrhs_here - 1)];
        }
        __syncthreads();
        double acc[NR];
#pragma unroll
        for (int c = 0; c < NR; ++c)
            acc[c] = 0.0;
#pragma unroll
        for (int cc = 0; cc < 16; ++cc)
#pragma unroll
            for (int c = 0; c < NR; ++c)
                acc[c] = __builtin_fma(m[cc], Y[(16 * q + cc) * NR + c], acc[c]);
#pragma unroll
        for (int c = 0; c < NR; ++c) {
            acc[c] += __shfl_xor(acc[c], 1);
            acc[c] += __shfl_xor(acc[c], 2);
        }
        if (q == 0) {
            if (solves) {
#pragma unroll
                for (int c = 0; c < 16; ++c)
                    Ys[rr * YP + c] = (c < NR && rr < rows && c < nrhs_here) ? bo[min(c, NR - 1)] - acc[min(c, NR - 1)]
                                                                            : 0.0;
            } else if (rr < rows) {
#pragma unroll
                for (int c = 0; c < NR; ++c)
                    if (c < nrhs_here)
                        B[(int64_t)(target * TB + rr) * ldb + c] = bo[c] - acc[c];
            }
        }
        __syncthreads();
    } else if (solves) {
        /* no update of the next block in this step: its rows as they are */
        const int b0 = next * TB;
        if (q == 0) {
            const double *brow = B + (int64_t)min(b0 + rr, n - 1) * ldb;
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                const double v = brow[min(c, nrhs_here - 1)];
                Ys[rr * YP + c] = (b0 + rr < n && c < nrhs_here) ? v : 0.0;
            }
        }
        __syncthreads();
    }
    if (solves)
        sky_pack_product<FWD>(pv, Ys, n, B, ldb, nrhs_here, next);
}

hipError_t skyline_pack(const SkyPlan &pl, const int32_t *f, const int64_t *rp, double *AL, const int32_t *g,
                        const int64_t *cp, double *AU, double *tiles, bool unpack, hipStream_t st)
{
    hipLaunchKernelGGL(k_sky_pack, dim3(2 * pl.nt), dim3(NT), 0, st, pl, f, rp, AL, g, cp, AU, tiles, unpack ? 1 : 0);
    return hipGetLastError();
}

template <int NR>
static hipError_t sky_sweeps(const SkyPlan &pl, const double *tiles, const double *P, double *B, int64_t ldb, int nh,
                             hipStream_t st)
{
    const int nt = pl.nt;
    /* forward: the launch for J = -1 solves block 0; the launch for J
     * updates the blocks below J from Y_J and solves block J + 1 */
    for (int J = -1; J + 1 < nt; ++J) {
        int cnt = 0;
        bool has_next = false;
        for (int R = J + 1; J >= 0 && R < nt; ++R)
            if (pl.F[R] <= J) {
                ++cnt;
                has_next |= R == J + 1;
            }
        hipLaunchKernelGGL((k_sky_sweep<NR, true>), dim3(cnt + (has_next ? 0 : 1)), dim3(NT), 0, st, pl, tiles, P,
                           B, ldb, nh, J, cnt);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    /* backward: the launch for J = nt solves block nt - 1; the launch for J
     * updates the blocks above J from X_J and solves block J - 1 */
    for (int J = nt; J > 0; --J) {
        const int cnt = J < nt ? J - pl.G[J] : 0;
        const bool has_next = J < nt && pl.G[J] <= J - 1;
        hipLaunchKernelGGL((k_sky_sweep<NR, false>), dim3(cnt + (has_next ? 0 : 1)), dim3(NT), 0, st, pl, tiles, P,
                           B, ldb, nh, J, cnt);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

hipError_t skyline_solve(const SkyPlan &pl, const double *tiles, double *P, double *B, int64_t ldb, int nrhs,
                         hipStream_t st)
{
    hipLaunchKernelGGL(k_sky_packs, dim3(pl.nt), dim3(NT), 0, st, pl, tiles, P);
    hipError_t e = hipGetLastError();
    for (int c0 = 0; c0 < nrhs && e == hipSuccess; c0 += 8) {
        const int nh = min(8, nrhs - c0);
        e = nh == 1 ? sky_sweeps<1>(pl, tiles, P, B + c0, ldb, nh, st)
            : nh <= 4 ? sky_sweeps<4>(pl, tiles, P, B + c0, ldb, nh, st)
                      : sky_sweeps<8>(pl, tiles, P, B + c0, ldb, nh, st);
    }
    return e;
}

/* ------------------------------------------------------------- adjoint --- */

/* Abar = -Bbar X^T for each system: coalesced row-major writes of the n x n
 * result; with one right-hand side each thread keeps its columns of x in
 * registers, otherwise the n x nrhs factors are read through the cache. */
template <typename T>
__global__ __launch_bounds__(NT) void k_outer_neg(int n, int nrhs, const T *__restrict__ Bb, int64_t ldb, int64_t strideB,
                                                  const T *__restrict__ X, int64_t ldx, int64_t strideX, T *__restrict__ Abar,
                                                  int64_t ldabar, int64_t strideAbar)
{
    const int sys = blockIdx.y;
    const T *bb = Bb + (int64_t)sys * strideB;
    const T *x = X + (int64_t)sys * strideX;
    T *ab = Abar + (int64_t)sys * strideAbar;
    if (nrhs == 1) {
        /* x in registers, 4 * NT columns at a time, for all the rows of the
         * workgroup: x is read once per workgroup rather than once per row
         * (the stream of writes evicts it from L2) */
        for (int j0 = 0; j0 < n; j0 += 4 * NT) {
            T xv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u)
                xv[u] = x[(int64_t)min(j0 + u * NT + (int)threadIdx.x, n - 1) * ldx];
            for (int i = blockIdx.x; i < n; i += gridDim.x) {
                const T bi = bb[(int64_t)i * ldb];
                T *row = ab + (int64_t)i * ldabar;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int j = j0 + u * NT + threadIdx.x;
                    if (j < n)
                        row[j] = -(bi * xv[u]);
                }
            }
        }
        return;
    }
    for (int i = blockIdx.x; i < n; i += gridDim.x)
        for (int j = threadIdx.x; j < n; j += NT) {
            T s = T(0);
            for (int c = 0; c < nrhs; ++c)
                s += bb[(int64_t)i * ldb + c] * x[(int64_t)j * ldx + c];
            ab[(int64_t)i * ldabar + j] = -s;
        }
}

template <typename T>
hipError_t outer_neg(int n, int nrhs, const T *Bb, int64_t ldb, int64_t strideB, const T *X, int64_t ldx,
                     int64_t strideX, T *Abar, int64_t ldabar, int64_t strideAbar, int64_t batch, hipStream_t st)
{
    for (int64_t b0 = 0; b0 < batch; b0 += 65535) {
        const int nb = (int)std::min<int64_t>(65535, batch - b0);
        const int gx = (int)std::min<int64_t>(n, std::max<int64_t>(1, 4096 / nb));
        hipLaunchKernelGGL(k_outer_neg<T>, dim3(gx, nb), dim3(NT), 0, st, n, nrhs, Bb + b0 * strideB, ldb, strideB,
                           X + b0 * strideX, ldx, strideX, Abar + b0 * strideAbar, ldabar, strideAbar);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

/* ----------------------------------------------------- mixed precision --- */

template <typename TI, typename TO>
__global__ void k_convert(int rows, int cols, const TI *__restrict__ S, int64_t lds, TO *__restrict__ D, int64_t ldd,
                          const int *skip)
{
    if (skip && *skip)
        return;
    const int64_t total = (int64_t)rows * cols;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / cols, j = e % cols;
        D[i * ldd + j] = (TO)S[i * lds + j];
    }
}

template <typename TI, typename TO>
hipError_t convert(int rows, int cols, const TI *S, int64_t lds, TO *D, int64_t ldd, const int *skip, hipStream_t st)
{
    const int64_t total = (int64_t)rows * cols;
    if (total <= 0)
        return hipSuccess;
    const int grid = (int)std::min<int64_t>((total + 255) / 256, 8192);
    hipLaunchKernelGGL((k_convert<TI, TO>), dim3(grid), dim3(256), 0, st, rows, cols, S, lds, D, ldd, skip);
    return hipGetLastError();
}

/* float(A) and the dominance margin, one wave per row: lanes split the row,
 * convert it and sum |a_ij| off the diagonal; the row's margin
 * |a_ii| - sum, clamped at 0, goes into *mbits by atomic minimum. */
__global__ __launch_bounds__(NT) void k_convert_margin(int n, const double *__restrict__ A, int64_t lda,
                                                       float *__restrict__ D, int64_t ldd, unsigned long long *mbits)
{
    const int l = threadIdx.x & 63;
    const int w = blockIdx.x * (NT / 64) + wave_id(), nw = gridDim.x * (NT / 64);
    double mloc = __longlong_as_double(0x7FF0000000000000ll);
    for (int i = w; i < n; i += nw) {
        const double *a = A + (int64_t)i * lda;
        float *d = D + (int64_t)i * ldd;
        double off = 0.0, dg = 0.0;
        for (int j = l; j < n; j += 64) {
            const double v = a[j];
            d[j] = (float)v;
            if (j == i)
                dg = fabs(v);
            else
                off += fabs(v);
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            off += __shfl_xor(off, o);
            dg += __shfl_xor(dg, o);
        }
        mloc = fmin(mloc, fmax(dg - off, 0.0));
    }
    if (l == 0)
        atomicMin(mbits, (unsigned long long)__double_as_longlong(mloc));
}

/* R = B - A X for NR <= 8 columns, one workgroup per row; max |r_ic| into bits[c]. */
template <int NR>
__global__ __launch_bounds__(NT) void k_residual(int n, int nrhs, const double *__restrict__ A, int64_t lda,
                                                 const double *__restrict__ B, int64_t ldb, const double *__restrict__ X,
                                                 int64_t ldx, double *__restrict__ R, int64_t ldr,
                                                 unsigned long long *bits, const int *skip)
{
    if (skip && *skip)
        return;
    __shared__ double red[4][NR];
    const int t = threadIdx.x;
    for (int i = blockIdx.x; i < n; i += gridDim.x) {
        double acc[NR];
#pragma unroll
        for (int c = 0; c < NR; ++c)
            acc[c] = 0.0;
        const double *ai = A + (int64_t)i * lda;
        for (int j = t; j < n; j += NT) {
            const double a = ai[j];
#pragma unroll
            for (int c = 0; c < NR; ++c)
                if (c < nrhs)
                    acc[c] += a * X[(int64_t)j * ldx + c];
        }
#pragma unroll
        for (int c = 0; c < NR; ++c) {
#pragma unroll
            for (int o = 32; o > 0; o >>= 1)
                acc[c] += __shfl_xor(acc[c], o);
        }
        if ((t & 63) == 0)
#pragma unroll
            for (int c = 0; c < NR; ++c)
                red[t >> 6][c] = acc[c];
        __syncthreads();
        if (t < nrhs && t < NR) {
            const double s = red[0][t] + red[1][t] + red[2][t] + red[3][t];
            const double r = B[(int64_t)i * ldb + t] - s;
            R[(int64_t)i * ldr + t] = r;
            atomicMax(bits + t, (unsigned long long)__double_as_longlong(fabs(r)));
        }
        __syncthreads();
    }
}

/* Stopping test after refinement step `it` (single thread).  With margin
 * m = min_i (|a_ii| - sum_{j != i} |a_ij|) > 0 the inverse is bounded,
 * ||A^{-1}||_inf <= 1/m, so the forward error of column c is at most
 * ||r_c||_inf / m; relative to the solution, ||r_c|| / (m ||x_c||). */
__global__ void k_check(int nrhs, unsigned long long *rbits, unsigned long long *xbits,
                        const unsigned long long *mbits, double tol, int it, int32_t *iters, double *ferr, int *conv)
{
    if (threadIdx.x != 0 || blockIdx.x != 0 || *conv)
        return;
    const double m = __longlong_as_double((long long)*mbits);
    bool all = true;
    for (int c = 0; c < nrhs; ++c) {
        const double r = __longlong_as_double((long long)rbits[c]);
        const double x = __longlong_as_double((long long)xbits[c]);
        const double den = m * x;
        const double bound = r == 0.0 ? 0.0 : (den > 0.0 ? r / den : __longlong_as_double(0x7FF0000000000000ll));
        if (ferr)
            ferr[c] = bound;
        if (bound <= tol) {
            if (iters && iters[c] < 0)
                iters[c] = it;
        } else {
            all = false;
        }
        rbits[c] = 0ull;
        xbits[c] = 0ull;
    }
    if (all)
        *conv = 1;
}

/* X (+)= D for the mixed-precision update; max |x_ic| of the result into xbits[c]. */
__global__ void k_xupdate(int n, int nrhs, double *__restrict__ X, int64_t ldx, const float *__restrict__ D,
                          int64_t ldd, int first, unsigned long long *xbits, const int *skip)
{
    if (skip && *skip)
        return;
    const int64_t total = (int64_t)n * nrhs;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / nrhs, c = e % nrhs;
        const double d = (double)D[i * ldd + c];
        const double x = first ? d : X[i * ldx + c] + d;
        X[i * ldx + c] = x;
        atomicMax(xbits + c, (unsigned long long)__double_as_longlong(fabs(x)));
    }
}

hipError_t convert_margin(int n, const double *A, int64_t lda, float *D, int64_t ldd, unsigned long long *mbits,
                          hipStream_t st)
{
    const int grid = std::max(1, std::min((n + 3) / 4, 4096));
    hipLaunchKernelGGL(k_convert_margin, dim3(grid), dim3(NT), 0, st, n, A, lda, D, ldd, mbits);
    return hipGetLastError();
}

hipError_t mixed_residual(int n, int nrhs, const double *A, int64_t lda, const double *B, int64_t ldb, const double *X,
                          int64_t ldx, double *R, int64_t ldr, unsigned long long *bits, const int *skip, hipStream_t st)
{
    const int grid = min(n, 16384);
    for (int c0 = 0; c0 < nrhs; c0 += 8) {
        const int nh = min(8, nrhs - c0);
        if (nh == 1)
            hipLaunchKernelGGL(k_residual<1>, dim3(grid), dim3(NT), 0, st, n, nh, A, lda, B + c0, ldb, X + c0, ldx,
                               R + c0, ldr, bits + c0, skip);
        else if (nh <= 4)
            hipLaunchKernelGGL(k_residual<4>, dim3(grid), dim3(NT), 0, st, n, nh, A, lda, B + c0, ldb, X + c0, ldx,
                               R + c0, ldr, bits + c0, skip);
        else
            hipLaunchKernelGGL(k_residual<8>, dim3(grid), dim3(NT), 0, st, n, nh, A, lda, B + c0, ldb, X + c0, ldx,
                               R + c0, ldr, bits + c0, skip);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

hipError_t mixed_check(int nrhs, unsigned long long *rbits, unsigned long long *xbits, const unsigned long long *mbits,
                       double tol, int it, int32_t *iters, double *ferr, int *conv, hipStream_t st)
{
    hipLaunchKernelGGL(k_check, dim3(1), dim3(64), 0, st, nrhs, rbits, xbits, mbits, tol, it, iters, ferr, conv);
    return hipGetLastError();
}

hipError_t mixed_xupdate(int n, int nrhs, double *X, int64_t ldx, const float *D, int64_t ldd, int first,
                         unsigned long long *xbits, const int *skip, hipStream_t st)
{
    const int64_t total = (int64_t)n * nrhs;
    const int grid = (int)std::min<int64_t>((total + 255) / 256, 4096);
    hipLaunchKernelGGL(k_xupdate, dim3(max(grid, 1)), dim3(256), 0, st, n, nrhs, X, ldx, D, ldd, first, xbits, skip);
    return hipGetLastError();
}

/* ------------------------------------------------ explicit instances --- */

template hipError_t dense_factor<double>(double *, int64_t, int, int32_t *, void *, const DenseTuning &, UpdateProfile *,
                                        hipStream_t, double *, int64_t, int, bool);
template hipError_t dense_factor<float>(float *, int64_t, int, int32_t *, void *, const DenseTuning &, UpdateProfile *,
                                       hipStream_t, float *, int64_t, int, bool);
template hipError_t factor_solve<double>(double *, int64_t, int, int32_t *, void *, const DenseTuning &, UpdateProfile *,
                                         hipStream_t, double *, int64_t, int);
template hipError_t factor_solve<float>(float *, int64_t, int, int32_t *, void *, const DenseTuning &, UpdateProfile *,
                                        hipStream_t, float *, int64_t, int);
template hipError_t dense_trsv<double>(int, const double *, int64_t, int, double *, int64_t, int, int *, double *,
                                       const int *, int32_t *, hipStream_t, bool, long long);
template hipError_t dense_trsv<float>(int, const float *, int64_t, int, float *, int64_t, int, int *, float *,
                                      const int *, int32_t *, hipStream_t, bool, long long);
template hipError_t batch_factor<double>(double *, int64_t, int, int64_t, int64_t, int32_t *, hipStream_t);
template hipError_t batch_factor<float>(float *, int64_t, int, int64_t, int64_t, int32_t *, hipStream_t);
template hipError_t batch_solve<double>(bool, const double *, int64_t, int, int64_t, double *, int64_t, int64_t, int, int64_t, hipStream_t);
template hipError_t batch_solve<float>(bool, const float *, int64_t, int, int64_t, float *, int64_t, int64_t, int, int64_t, hipStream_t);
template hipError_t batched_run<double>(int, const int *, const int64_t *, double *, const int64_t *, double *, const int *, int32_t *, int *, int, hipStream_t);
template hipError_t batched_run<float>(int, const int *, const int64_t *, float *, const int64_t *, float *, const int *, int32_t *, int *, int, hipStream_t);
template hipError_t lu_inverse<double>(const double *, int64_t, int, double *, int64_t, double *, hipStream_t);
template hipError_t lu_inverse<float>(const float *, int64_t, int, float *, int64_t, float *, hipStream_t);
template hipError_t outer_neg<double>(int, int, const double *, int64_t, int64_t, const double *, int64_t, int64_t, double *, int64_t, int64_t, int64_t, hipStream_t);
template hipError_t outer_neg<float>(int, int, const float *, int64_t, int64_t, const float *, int64_t, int64_t, float *, int64_t, int64_t, int64_t, hipStream_t);
template hipError_t convert<double, float>(int, int, const double *, int64_t, float *, int64_t, const int *, hipStream_t);
template hipError_t convert<float, double>(int, int, const float *, int64_t, double *, int64_t, const int *, hipStream_t);

} /* namespace ebv */
