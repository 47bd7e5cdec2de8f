/*
 * HIP kernels and their launchers for libebv (gfx950).
 *
 * Dense single system (Eq. 6-a/6-c applied 64 steps at a time):
 *   k_panel   factors the 64x64 diagonal tile and, in the same launch, the U
 *             blocks right of it and the L blocks below it;
 *   k_update  applies the rank-64 trailing update on the matrix cores.
 * Triangular solves (Eq. 1): k_trsv, one workgroup per 64-row block,
 *   workgroups take blocks in solve order from a ticket counter and wait for
 *   the blocks they depend on through per-block flags (no grid barrier).
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

/* ------------------------------------------------------- dense factor --- */

/*
 * Diagonal tile of a panel step: factor the 64x64 tile at (d0, d0) in
 * registers and store it in place for the triangular solves of the next
 * launch.  Called by the single workgroup of k_diag (the first step) and by
 * the extra workgroup of k_update (every later step).
 */
template <typename T>
__device__ __forceinline__ void diag_tile(T *__restrict__ A, int64_t lda, int n, int d0, int32_t *info,
                                          TileSmem<T> &sm)
{
    const int dw = min(TB, n - d0);
    T *Add = A + (int64_t)d0 * lda + d0;
    T a[4][4];
    rt_load(a, Add, lda, dw, dw, true);
    const int z = rt_lu(a, sm, dw);
    rt_store(a, Add, lda, dw, dw);
    if (threadIdx.x == 0 && info && z && *info == 0)
        *info = d0 + z;
}

template <typename T>
__global__ __launch_bounds__(NT) void k_diag(T *__restrict__ A, int64_t lda, int n, int d0, int32_t *info)
{
    __shared__ TileSmem<T> sm;
    diag_tile(A, lda, n, d0, info, sm);
}

/*
 * Triangular solves of one panel step.  The diagonal tile was factored in
 * place by the previous launch; each workgroup stages it in LDS and solves
 * one 64x64 block against it: a U block right of it (U_kj = L_kk^{-1} A_kj)
 * or an L block below it (L_ik = A_ik U_kk^{-1}).
 */
template <typename T>
__global__ __launch_bounds__(NT) void k_panel(T *__restrict__ A, int64_t lda, int n, int k0)
{
    __shared__ TileSmem<T> sm;
    const int kw = min(TB, n - k0);
    const int nrem = (n - k0 - kw + TB - 1) / TB;
    const int t = blockIdx.x;
    stage64<T, false>(sm.t0, A + (int64_t)k0 * lda + k0, lda, kw, kw);
    __syncthreads();
    if (threadIdx.x < TB)
        sm.rinv[threadIdx.x] = recip(sm.t0[threadIdx.x * LDT + threadIdx.x]);
    __syncthreads();
    T x[4][4];
    if (t < nrem) {
        const int j0 = k0 + kw + t * TB, jw = min(TB, n - j0);
        T *G = A + (int64_t)k0 * lda + j0;
        rt_load(x, G, lda, kw, jw, false);
        rt_trsm_lower_unit(x, sm.t0, sm);
        rt_store(x, G, lda, kw, jw);
    } else {
        const int i0 = k0 + kw + (t - nrem) * TB, iw = min(TB, n - i0);
        T *G = A + (int64_t)i0 * lda + k0;
        rt_load(x, G, lda, iw, kw, false);
        rt_trsm_upper_right(x, sm.t0, sm.rinv, sm);
        rt_store(x, G, lda, iw, kw);
    }
}

/*
 * Trailing update A22 -= L21 U12 for one block step (K = kw <= 64): the
 * rank-kw update of Eq. 6-c on the matrix cores.  Each workgroup owns a
 * BM x BN tile of A22 held in registers for the whole K loop (read once,
 * written once); 4 waves, each a (BM/2) x (BN/2) block of 16x16 matrix-core
 * tiles.  K runs in BK-deep chunks through double-buffered LDS: the next
 * chunk's global loads are in flight while the current one feeds the matrix
 * cores.  L21 is kept row-major in LDS with an odd pitch (conflict-free
 * column reads), U12 row-major.  Tiles are dealt to the 8 XCDs in contiguous
 * runs (workgroups are dispatched round-robin over XCDs), so neighbouring
 * tiles share an XCD's L2.
 */
template <typename T, int BM, int BN, int BK>
__global__ __launch_bounds__(NT, 2) void k_update(T *__restrict__ A, int64_t lda, int n, int k0, int kw,
                                                  int32_t *info)
{
    typedef typename vec4<T>::type V;
    constexpr int WM = BM / 2, WN = BN / 2, MB = WM / 16, NB = WN / 16;
    constexpr int PA = BK + 1, PB = BN + 4;
    constexpr int EA = BM * BK / NT, EB = BK * BN / NT; /* elements per thread per chunk */
    static_assert(BK % EA == 0 && BN % EB == 0, "chunk split");
    constexpr size_t GEMM_LDS = sizeof(T) * 2 * (BM * PA + BK * PB);
    constexpr size_t LDS_BYTES = GEMM_LDS > sizeof(TileSmem<T>) ? GEMM_LDS : sizeof(TileSmem<T>);
    __shared__ __attribute__((aligned(16))) char lds_raw[LDS_BYTES];
    T(*sA)[BM * PA] = reinterpret_cast<T(*)[BM * PA]>(lds_raw);
    T(*sB)[BK * PB] = reinterpret_cast<T(*)[BK * PB]>(lds_raw + sizeof(T) * 2 * BM * PA);

    const int i0 = k0 + kw, m = n - i0;
    const int tiles_n = (m + BN - 1) / BN;
    const int ntiles = ((m + BM - 1) / BM) * tiles_n;
    const int b = blockIdx.x;
    const int dw = min(TB, m); /* next diagonal tile: rows/cols i0..i0+dw */
    if (b == ntiles) {
        /* the extra workgroup: update the next diagonal tile itself and factor
         * it in place (the next panel step's diagonal tile); the tile
         * workgroup covering it does not store that corner */
        TileSmem<T> &sm = *reinterpret_cast<TileSmem<T> *>(lds_raw);
        stage64<T, true>(sm.t0, A + (int64_t)i0 * lda + k0, lda, dw, kw);
        stage64<T, false>(sm.t1, A + (int64_t)k0 * lda + i0, lda, kw, dw);
        __syncthreads();
        wg_gemm64(DenseC<T>{A + (int64_t)i0 * lda + i0, lda, dw, dw}, sm.t0, sm.t1);
        __syncthreads();
        diag_tile(A, lda, n, i0, info, sm);
        return;
    }
    const int xcd = b & 7, per = ntiles >> 3, rem = ntiles & 7;
    const int tile = xcd * per + min(xcd, rem) + (b >> 3);
    const int r0 = i0 + (tile / tiles_n) * BM, c0 = i0 + (tile % tiles_n) * BN;
    const int nr = min(BM, n - r0), nc = min(BN, n - c0);
    const bool corner = r0 == i0 && c0 == i0; /* holds the next diagonal tile */

    const int t = threadIdx.x, w = t >> 6, l = t & 63, lr = l & 15, lk = l >> 4;
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
                if (row < nr && col < nc && !(corner && row < dw && col < dw))
                    A[(int64_t)(r0 + row) * lda + c0 + col] = acc[bi][bj][r];
            }
}

/* ----------------------------------------- update-kernel measurement --- */

/* When enabled, dense_factor brackets every k_update launch with a pair of
 * events (created up front) and records the launch's algorithmic flop count
 * 2 * m * m * kw, so that the caller can report the kernel's live average
 * duration and achieved rate. */
namespace {
struct UpdateProfile {
    std::vector<hipEvent_t> ev;
    std::vector<double> flops;
    int used = 0;
} g_prof;
} // namespace

int profile_update_enable(int max_launches)
{
    for (hipEvent_t e : g_prof.ev)
        (void)hipEventDestroy(e);
    g_prof.ev.clear();
    g_prof.flops.clear();
    g_prof.used = 0;
    if (max_launches <= 0)
        return 0;
    g_prof.ev.resize(2 * (size_t)max_launches);
    g_prof.flops.resize((size_t)max_launches);
    for (hipEvent_t &e : g_prof.ev)
        if (hipEventCreate(&e) != hipSuccess)
            return 1;
    return 0;
}

int profile_update_read(double *ms_total, int64_t *launches, double *flops_total)
{
    double ms = 0.0, fl = 0.0;
    for (int i = 0; i < g_prof.used; ++i) {
        if (hipEventSynchronize(g_prof.ev[2 * i + 1]) != hipSuccess)
            return 1;
        float t = 0.f;
        if (hipEventElapsedTime(&t, g_prof.ev[2 * i], g_prof.ev[2 * i + 1]) != hipSuccess)
            return 1;
        ms += t;
        fl += g_prof.flops[i];
    }
    *ms_total = ms;
    *launches = g_prof.used;
    *flops_total = fl;
    g_prof.used = 0;
    return 0;
}

static bool profile_slot(hipStream_t st, double flops, int &slot)
{
    if (g_prof.used >= (int)g_prof.flops.size())
        return false;
    slot = g_prof.used++;
    g_prof.flops[slot] = flops;
    (void)hipEventRecord(g_prof.ev[2 * slot], st);
    return true;
}

template <typename T>
hipError_t dense_factor(T *A, int64_t lda, int n, int32_t *info, void *slot_ws, const DenseTuning &tun,
                        hipStream_t st)
{
    (void)slot_ws;
    hipError_t e = hipSuccess;
    if (info) {
        e = fill_i32(info, 1, 0, st);
        if (e != hipSuccess)
            return e;
    }
    hipLaunchKernelGGL(k_diag<T>, dim3(1), dim3(NT), 0, st, A, lda, n, 0, info);
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    for (int k0 = 0; k0 < n; k0 += TB) {
        const int kw = min(TB, n - k0);
        const int nrem = (n - k0 - kw + TB - 1) / TB;
        if (nrem == 0)
            break;
        hipLaunchKernelGGL(k_panel<T>, dim3(2 * nrem), dim3(NT), 0, st, A, lda, n, k0);
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
        const int m = n - k0 - kw;
        int pslot = -1;
        const bool prof = profile_slot(st, 2.0 * (double)m * (double)m * (double)kw, pslot);
        if (m > tun.small_update_below) {
            const int nt = ((m + 127) / 128) * ((m + 127) / 128);
            hipLaunchKernelGGL((k_update<T, 128, 128, 16>), dim3(nt + 1), dim3(NT), 0, st, A, lda, n, k0, kw, info);
        } else {
            const int nt = ((m + 63) / 64) * ((m + 63) / 64);
            hipLaunchKernelGGL((k_update<T, 64, 64, 16>), dim3(nt + 1), dim3(NT), 0, st, A, lda, n, k0, kw, info);
        }
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
        if (prof)
            (void)hipEventRecord(g_prof.ev[2 * pslot + 1], st);
    }
    return e;
}

/* ------------------------------------------------- triangular solves --- */

template <typename T, int MODE, int NR>
__global__ __launch_bounds__(NT) void k_trsv(const T *__restrict__ LU, int64_t lda, int n, T *__restrict__ B,
                                             int64_t ldb, int nrhs_here, int *wsi, const int *skip)
{
    if (skip && *skip)
        return;
    __shared__ TileSmem<T> sm;
    int *status = wsi, *ctr = wsi + 1, *flags = wsi + 2;
    if (threadIdx.x == 0)
        sm.ticket = atomicAdd(ctr, 1);
    __syncthreads();
    const int nb = (n + TB - 1) / TB;
    if (sm.ticket >= nb) { /* counter not reset: refuse rather than index out of range */
        if (threadIdx.x == 0)
            atomicOr(status, 2);
        return;
    }
    const int blk = tri_forward(MODE) ? sm.ticket : nb - 1 - sm.ticket;
    const DenseOp<T, MODE> op{LU, lda, n};
    solve_block<T, MODE, NR>(op, n, B, ldb, nrhs_here, blk, nb, sm, flags, status);
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0)
        __hip_atomic_store(flags + blk, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T, int MODE>
static hipError_t trsv_mode(const T *LU, int64_t lda, int n, T *B, int64_t ldb, int nrhs, int *wsi,
                            const int *skip, hipStream_t st)
{
    const int nb = (n + TB - 1) / TB;
    hipError_t e = hipSuccess;
    for (int c0 = 0; c0 < nrhs; c0 += 8) {
        const int nh = min(8, nrhs - c0);
        if ((e = fill_i32(wsi + 1, 1 + nb, 0, st)) != hipSuccess)
            return e;
        if (nh == 1)
            hipLaunchKernelGGL((k_trsv<T, MODE, 1>), dim3(nb), dim3(NT), 0, st, LU, lda, n, B + c0, ldb, nh, wsi, skip);
        else if (nh == 2)
            hipLaunchKernelGGL((k_trsv<T, MODE, 2>), dim3(nb), dim3(NT), 0, st, LU, lda, n, B + c0, ldb, nh, wsi, skip);
        else if (nh <= 4)
            hipLaunchKernelGGL((k_trsv<T, MODE, 4>), dim3(nb), dim3(NT), 0, st, LU, lda, n, B + c0, ldb, nh, wsi, skip);
        else
            hipLaunchKernelGGL((k_trsv<T, MODE, 8>), dim3(nb), dim3(NT), 0, st, LU, lda, n, B + c0, ldb, nh, wsi, skip);
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
    }
    return e;
}

template <typename T>
hipError_t dense_trsv(int mode, const T *LU, int64_t lda, int n, T *B, int64_t ldb, int nrhs, int *wsi,
                      const int *skip, hipStream_t st)
{
    switch (mode) {
    case TRI_L: return trsv_mode<T, TRI_L>(LU, lda, n, B, ldb, nrhs, wsi, skip, st);
    case TRI_U: return trsv_mode<T, TRI_U>(LU, lda, n, B, ldb, nrhs, wsi, skip, st);
    case TRI_UT: return trsv_mode<T, TRI_UT>(LU, lda, n, B, ldb, nrhs, wsi, skip, st);
    default: return trsv_mode<T, TRI_LT>(LU, lda, n, B, ldb, nrhs, wsi, skip, st);
    }
}

/* ---------------------------------------------------- uniform batches --- */

template <typename T>
__global__ __launch_bounds__(NT) void k_lu_batch(T *__restrict__ A, int64_t lda, int n, int64_t strideA,
                                                    int32_t *info)
{
    __shared__ TileSmem<T> sm;
    T *Ab = A + (int64_t)blockIdx.x * strideA;
    const int z = wg_lu(Ab, lda, n, sm);
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
            if (nh == 1)
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
__global__ __launch_bounds__(NT) void k_batched(int count, const int *__restrict__ ns, const int64_t *__restrict__ offA,
                                                   T *__restrict__ A, const int64_t *__restrict__ offB, T *__restrict__ B,
                                                   const int *__restrict__ order, int32_t *info, int *queue)
{
    __shared__ TileSmem<T> sm;
    for (;;) {
        if (threadIdx.x == 0)
            sm.ticket = atomicAdd(queue, 1);
        __syncthreads();
        const int idx = sm.ticket;
        __syncthreads();
        if (idx >= count)
            break;
        const int s = order ? order[idx] : idx;
        const int n = ns[s];
        if (n <= 0) {
            if (threadIdx.x == 0 && info)
                info[s] = 0;
            continue;
        }
        T *As = A + offA[s];
        const int z = wg_lu(As, n, n, sm);
        if (threadIdx.x == 0 && info)
            info[s] = z;
        if (B) {
            T *Bs = B + offB[s];
            wg_solve<T, TRI_L, 1>(As, n, n, Bs, 1, 1, sm);
            wg_solve<T, TRI_U, 1>(As, n, n, Bs, 1, 1, sm);
        }
    }
}

/* Workgroup-wide max of a non-negative value (result valid in every thread). */
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
 * update x += solve_float(r), stop at max|r| / max|b| <= tol). */
__global__ __launch_bounds__(NT) void k_batched_mixed(int count, const int *__restrict__ ns, const int64_t *__restrict__ offA,
                                                         const double *__restrict__ A, const int64_t *__restrict__ offB,
                                                         double *__restrict__ B, const int *__restrict__ order,
                                                         int32_t *info, int *queue, float *__restrict__ W,
                                                         float *__restrict__ R32, double *__restrict__ X,
                                                         int max_iter, double tol, int32_t *iters)
{
    __shared__ TileSmem<float> sm;
    __shared__ double red[4];
    const int t = threadIdx.x, w = t >> 6, l = t & 63;
    for (;;) {
        if (t == 0)
            sm.ticket = atomicAdd(queue, 1);
        __syncthreads();
        const int idx = sm.ticket;
        __syncthreads();
        if (idx >= count)
            break;
        const int s = order ? order[idx] : idx;
        const int n = ns[s];
        if (n <= 0) {
            if (t == 0) {
                if (info)
                    info[s] = 0;
                if (iters)
                    iters[s] = 0;
            }
            continue;
        }
        const double *As = A + offA[s];
        double *bs = B + offB[s];
        float *Ws = W + offA[s];
        float *rs = R32 + offB[s];
        double *xs = X + offB[s];
        const int64_t nn = (int64_t)n * n;
        for (int64_t i = t; i < nn; i += NT)
            Ws[i] = (float)As[i];
        double bmax = 0.0;
        for (int i = t; i < n; i += NT) {
            rs[i] = (float)bs[i];
            bmax = fmax(bmax, fabs(bs[i]));
        }
        bmax = wg_max(bmax, red);
        __syncthreads();
        const int z = wg_lu(Ws, n, n, sm);
        if (t == 0 && info)
            info[s] = z;
        int used = -1;
        for (int it = 0; it <= max_iter; ++it) {
            wg_solve<float, TRI_L, 1>(Ws, n, n, rs, 1, 1, sm);
            wg_solve<float, TRI_U, 1>(Ws, n, n, rs, 1, 1, sm);
            for (int i = t; i < n; i += NT)
                xs[i] = (it == 0) ? (double)rs[i] : xs[i] + (double)rs[i];
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
            if (rmax <= tol * bmax) {
                used = it;
                break;
            }
        }
        __syncthreads();
        for (int i = t; i < n; i += NT)
            bs[i] = xs[i];
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

/* Row-wise band storage: a_ij at AB[i*ldab + j - i + kl] for -kl <= j - i <= ku. */
struct BandRef {
    double *AB;
    int64_t ldab;
    int n, kl, ku;
    __device__ __forceinline__ double *at(int i, int j) const
    {
        const int d = j - i;
        return (i >= 0 && j >= 0 && i < n && j < n && d >= -kl && d <= ku) ? AB + (int64_t)i * ldab + (d + kl) : nullptr;
    }
};

/* Tile (r0.., c0..) of a band matrix as a wg_gemm64 accessor. */
struct BandTileC {
    BandRef br;
    int r0, c0;
    __device__ __forceinline__ double *operator()(int r, int c) const { return br.at(r0 + r, c0 + c); }
};

/* Register-tile load/store of block (r0, c0) of a band matrix (zero outside
 * the band; identity padding past the matrix end when pad_identity). */
__device__ __forceinline__ void band_rt_load(double (&a)[4][4], const BandRef &br, int r0, int c0, bool pad_identity)
{
    const int tr = threadIdx.x >> 4, tc = threadIdx.x & 15;
#pragma unroll
    for (int qr = 0; qr < 4; ++qr)
#pragma unroll
        for (int qc = 0; qc < 4; ++qc) {
            const int i = trow(tr, qr), j = trow(tc, qc);
            const double *p = br.at(r0 + i, c0 + j);
            a[qr][qc] = p ? *p : ((pad_identity && i == j && r0 + i >= br.n) ? 1.0 : 0.0);
        }
}
__device__ __forceinline__ void band_rt_store(const double (&a)[4][4], const BandRef &br, int r0, int c0)
{
    const int tr = threadIdx.x >> 4, tc = threadIdx.x & 15;
#pragma unroll
    for (int qr = 0; qr < 4; ++qr)
#pragma unroll
        for (int qc = 0; qc < 4; ++qc) {
            double *p = br.at(r0 + trow(tr, qr), c0 + trow(tc, qc));
            if (p)
                *p = a[qr][qc];
        }
}

/*
 * Band Doolittle LU by one workgroup.  With kl, ku <= 64 the matrix is block
 * tridiagonal in 64x64 tiles and, without pivoting, so are its factors: each
 * block step factors the diagonal tile, solves the one U tile to its right and
 * the one L tile below it, and updates the next diagonal tile on the matrix
 * cores.  Entries outside the band stay exactly zero and are never stored.
 */
__global__ __launch_bounds__(NT) void k_band_factor(double *AB, int64_t ldab, int n, int kl, int ku, int32_t *info)
{
    __shared__ TileSmem<double> sm;
    const BandRef br{AB, ldab, n, kl, ku};
    const int nt = (n + TB - 1) / TB;
    const int tr = threadIdx.x >> 4, tc = threadIdx.x & 15;
    int zero_at = 0;
    double a[4][4];
    for (int kb = 0; kb < nt; ++kb) {
        const int k0 = kb * TB, kw = min(TB, n - k0);
        band_rt_load(a, br, k0, k0, true);
        const int z = rt_lu(a, sm, kw);
        if (z && !zero_at)
            zero_at = k0 + z;
        band_rt_store(a, br, k0, k0);
        if (kb + 1 == nt)
            break;
        rt_store_lds(a, sm.t0);
        __syncthreads();
        const int k1 = k0 + TB;
        band_rt_load(a, br, k0, k1, false);
        rt_trsm_lower_unit(a, sm.t0, sm);
        band_rt_store(a, br, k0, k1);
        rt_store_lds(a, sm.t1); /* U12: the B operand of the update */
        band_rt_load(a, br, k1, k0, false);
        rt_trsm_upper_right(a, sm.t0, sm.rinv, sm);
        band_rt_store(a, br, k1, k0);
#pragma unroll
        for (int qr = 0; qr < 4; ++qr) /* L21 transposed: the A operand */
#pragma unroll
            for (int qc = 0; qc < 4; ++qc)
                sm.t0[trow(tc, qc) * LDT + trow(tr, qr)] = a[qr][qc];
        __syncthreads();
        wg_gemm64(BandTileC{br, k1, k1}, sm.t0, sm.t1);
        __syncthreads();
    }
    if (threadIdx.x == 0 && info)
        *info = zero_at;
}

/* Operator tiles of the band factor for the solves. */
template <int MODE> struct BandOp {
    BandRef br;
    __device__ __forceinline__ void operator()(double *S, int bi, int bj) const
    {
        for (int idx = threadIdx.x; idx < TB * TB; idx += NT) {
            const int r = idx >> 6, c = idx & 63;
            const double *p = br.at(bi * TB + r, bj * TB + c);
            S[r * LDT + c] = p ? *p : 0.0;
        }
    }
    __device__ __forceinline__ void seg(int bi, int bj, int rr, int q, double (&m)[16]) const
    {
#pragma unroll
        for (int cc = 0; cc < 16; ++cc) {
            const double *p = br.at(bi * TB + rr, bj * TB + 16 * q + cc);
            m[cc] = p ? *p : 0.0;
        }
    }
};

template <int NR>
__global__ __launch_bounds__(NT) void k_band_solve(const double *AB, int64_t ldab, int n, int kl, int ku, double *B,
                                                   int64_t ldb, int nrhs_here)
{
    __shared__ TileSmem<double> sm;
    const BandRef br{const_cast<double *>(AB), ldab, n, kl, ku};
    const int nb = (n + TB - 1) / TB;
    const BandOp<TRI_L> opl{br};
    const BandOp<TRI_U> opu{br};
    for (int s = 0; s < nb; ++s)
        solve_block<double, TRI_L, NR>(opl, n, B, ldb, nrhs_here, s, 1, sm, nullptr, nullptr);
    for (int s = 0; s < nb; ++s)
        solve_block<double, TRI_U, NR>(opu, n, B, ldb, nrhs_here, nb - 1 - s, 1, sm, nullptr, nullptr);
}

hipError_t band_factor(double *AB, int64_t ldab, int n, int kl, int ku, int32_t *info, hipStream_t st)
{
    hipLaunchKernelGGL(k_band_factor, dim3(1), dim3(NT), 0, st, AB, ldab, n, kl, ku, info);
    return hipGetLastError();
}

hipError_t band_solve(const double *AB, int64_t ldab, int n, int kl, int ku, double *B, int64_t ldb, int nrhs,
                      hipStream_t st)
{
    for (int c0 = 0; c0 < nrhs; c0 += 8) {
        const int nh = min(8, nrhs - c0);
        if (nh == 1)
            hipLaunchKernelGGL(k_band_solve<1>, dim3(1), dim3(NT), 0, st, AB, ldab, n, kl, ku, B + c0, ldb, nh);
        else if (nh <= 4)
            hipLaunchKernelGGL(k_band_solve<4>, dim3(1), dim3(NT), 0, st, AB, ldab, n, kl, ku, B + c0, ldb, nh);
        else
            hipLaunchKernelGGL(k_band_solve<8>, dim3(1), dim3(NT), 0, st, AB, ldab, n, kl, ku, B + c0, ldb, nh);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

/* ------------------------------------------------------------- adjoint --- */

/* Abar = -Bbar X^T for each system: coalesced row-major writes of the n x n
 * result, the n x nrhs factors read through the cache. */
template <typename T>
__global__ __launch_bounds__(NT) void k_outer_neg(int n, int nrhs, const T *__restrict__ Bb, int64_t ldb, int64_t strideB,
                                                  const T *__restrict__ X, int64_t ldx, int64_t strideX, T *__restrict__ Abar,
                                                  int64_t ldabar, int64_t strideAbar)
{
    const int sys = blockIdx.y;
    const T *bb = Bb + (int64_t)sys * strideB;
    const T *x = X + (int64_t)sys * strideX;
    T *ab = Abar + (int64_t)sys * strideAbar;
    for (int i = blockIdx.x; i < n; i += gridDim.x) {
        if (nrhs == 1) {
            const T bi = bb[(int64_t)i * ldb];
            for (int j = threadIdx.x; j < n; j += NT)
                ab[(int64_t)i * ldabar + j] = -(bi * x[(int64_t)j * ldx]);
        } else {
            for (int j = threadIdx.x; j < n; j += NT) {
                T s = T(0);
                for (int c = 0; c < nrhs; ++c)
                    s += bb[(int64_t)i * ldb + c] * x[(int64_t)j * ldx + c];
                ab[(int64_t)i * ldabar + j] = -s;
            }
        }
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

/* Column max |B_ic| into bits[c] (non-negative doubles order like their bit patterns). */
__global__ void k_colmax(int n, int nrhs, const double *__restrict__ B, int64_t ldb, unsigned long long *bits)
{
    for (int c = 0; c < nrhs; ++c) {
        double m = 0.0;
        for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
            m = fmax(m, fabs(B[(int64_t)i * ldb + c]));
#pragma unroll
        for (int o = 32; o > 0; o >>= 1)
            m = fmax(m, __shfl_xor(m, o));
        if ((threadIdx.x & 63) == 0)
            atomicMax(bits + c, (unsigned long long)__double_as_longlong(m));
    }
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

/* Stopping test after refinement step `it` (single thread). */
__global__ void k_check(int nrhs, unsigned long long *rbits, const unsigned long long *bbits, double tol, int it,
                        int32_t *iters, double *relres, int *conv)
{
    if (threadIdx.x != 0 || blockIdx.x != 0 || *conv)
        return;
    bool all = true;
    for (int c = 0; c < nrhs; ++c) {
        const double r = __longlong_as_double((long long)rbits[c]);
        const double b = __longlong_as_double((long long)bbits[c]);
        const double rel = b > 0.0 ? r / b : r;
        if (relres)
            relres[c] = rel;
        if (rel <= tol) {
            if (iters && iters[c] < 0)
                iters[c] = it;
        } else {
            all = false;
        }
        rbits[c] = 0ull;
    }
    if (all)
        *conv = 1;
}

/* X (+)= D for the mixed-precision update. */
__global__ void k_xupdate(int n, int nrhs, double *__restrict__ X, int64_t ldx, const float *__restrict__ D,
                          int64_t ldd, int first, const int *skip)
{
    if (skip && *skip)
        return;
    const int64_t total = (int64_t)n * nrhs;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / nrhs, c = e % nrhs;
        const double d = (double)D[i * ldd + c];
        X[i * ldx + c] = first ? d : X[i * ldx + c] + d;
    }
}

hipError_t mixed_colmax(int n, int nrhs, const double *B, int64_t ldb, unsigned long long *bits, hipStream_t st)
{
    hipLaunchKernelGGL(k_colmax, dim3(min(1024, (n + 255) / 256)), dim3(256), 0, st, n, nrhs, B, ldb, bits);
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

hipError_t mixed_check(int nrhs, unsigned long long *rbits, const unsigned long long *bbits, double tol, int it,
                       int32_t *iters, double *relres, int *conv, hipStream_t st)
{
    hipLaunchKernelGGL(k_check, dim3(1), dim3(64), 0, st, nrhs, rbits, bbits, tol, it, iters, relres, conv);
    return hipGetLastError();
}

hipError_t mixed_xupdate(int n, int nrhs, double *X, int64_t ldx, const float *D, int64_t ldd, int first,
                         const int *skip, hipStream_t st)
{
    const int64_t total = (int64_t)n * nrhs;
    const int grid = (int)std::min<int64_t>((total + 255) / 256, 4096);
    hipLaunchKernelGGL(k_xupdate, dim3(max(grid, 1)), dim3(256), 0, st, n, nrhs, X, ldx, D, ldd, first, skip);
    return hipGetLastError();
}

/* ------------------------------------------------ explicit instances --- */

template hipError_t dense_factor<double>(double *, int64_t, int, int32_t *, void *, const DenseTuning &, hipStream_t);
template hipError_t dense_factor<float>(float *, int64_t, int, int32_t *, void *, const DenseTuning &, hipStream_t);
template hipError_t dense_trsv<double>(int, const double *, int64_t, int, double *, int64_t, int, int *, const int *, hipStream_t);
template hipError_t dense_trsv<float>(int, const float *, int64_t, int, float *, int64_t, int, int *, const int *, hipStream_t);
template hipError_t batch_factor<double>(double *, int64_t, int, int64_t, int64_t, int32_t *, hipStream_t);
template hipError_t batch_factor<float>(float *, int64_t, int, int64_t, int64_t, int32_t *, hipStream_t);
template hipError_t batch_solve<double>(bool, const double *, int64_t, int, int64_t, double *, int64_t, int64_t, int, int64_t, hipStream_t);
template hipError_t batch_solve<float>(bool, const float *, int64_t, int, int64_t, float *, int64_t, int64_t, int, int64_t, hipStream_t);
template hipError_t batched_run<double>(int, const int *, const int64_t *, double *, const int64_t *, double *, const int *, int32_t *, int *, int, hipStream_t);
template hipError_t batched_run<float>(int, const int *, const int64_t *, float *, const int64_t *, float *, const int *, int32_t *, int *, int, hipStream_t);
template hipError_t outer_neg<double>(int, int, const double *, int64_t, int64_t, const double *, int64_t, int64_t, double *, int64_t, int64_t, int64_t, hipStream_t);
template hipError_t outer_neg<float>(int, int, const float *, int64_t, int64_t, const float *, int64_t, int64_t, float *, int64_t, int64_t, int64_t, hipStream_t);
template hipError_t convert<double, float>(int, int, const double *, int64_t, float *, int64_t, const int *, hipStream_t);
template hipError_t convert<float, double>(int, int, const float *, int64_t, double *, int64_t, const int *, hipStream_t);

} /* namespace ebv */
