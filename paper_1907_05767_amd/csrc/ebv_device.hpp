/*
 * Device building blocks for the EbV LU kernels (gfx950, wave64).
 *
 * Every routine here is executed by a whole 256-thread workgroup (4 waves).
 *
 * Register tiles.  A 64 x 64 tile is held in registers, 16 values per thread:
 * thread t = 16*tr + tc owns rows ebv_row(tr, q) and columns ebv_row(tc, q),
 * q = 0..3, i.e. the EbV-joined row pairs {v, 63-v} (and likewise columns).
 * One elimination step k (Eq. 6-a, 6-c) then costs every thread the same
 * number of multiply-adds to within one row/column of the mean, which is the
 * equal-work property the paper's equalization is after.
 *
 * Each step publishes the pivot row and the pivot column through LDS (the
 * "shared memory" the paper stages through), double-buffered so that one
 * barrier per step suffices.
 */
#ifndef EBV_DEVICE_HPP
#define EBV_DEVICE_HPP

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ebv_pairing.h"

namespace ebv {

constexpr int TB = 64;     /* tile edge */
constexpr int NT = 256;    /* threads per workgroup */
constexpr int LDT = TB + 1;/* LDS row pitch of a staged tile (odd: spreads banks) */

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T> struct vec4;
template <> struct vec4<double> { typedef d4 type; };
template <> struct vec4<float> { typedef f4 type; };

/* 16x16x4 matrix-core step: D = A(16x4) * B(4x16) + C.
 * Lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]; element r of the
 * result is D[acc_row<T>(l / 16, r)][l % 16].  The two precisions place the
 * rows differently (measured on gfx950): the double form interleaves them,
 * row l/16 + 4r; the float form keeps them contiguous, row 4*(l/16) + r. */
__device__ __forceinline__ d4 mfma16(double a, double b, d4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma16(float a, float b, f4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
template <typename T> __device__ __forceinline__ constexpr int acc_row(int lk, int r);
template <> __device__ __forceinline__ constexpr int acc_row<double>(int lk, int r) { return lk + 4 * r; }
template <> __device__ __forceinline__ constexpr int acc_row<float>(int lk, int r) { return 4 * lk + r; }

__device__ __forceinline__ int trow(int u, int q) { return ebv_row(u, q, 16, TB); }

/* -------------------------------------------------------- LDS layouts --- */

/* Scratch shared by the tile routines of one workgroup. */
template <typename T> struct TileSmem {
    union {
        struct {               /* factored diagonal tile and its pivot reciprocals */
            T D[TB * LDT];
            T rinv[TB];
        } d;
        struct {               /* matrix-core operands: A transposed, B as is */
            T AT[TB * LDT];
            T B[TB * LDT];
        } g;
        struct {               /* triangular solve: tile + a published block of X */
            T M[TB * LDT];
            T Y[TB * 8];
        } s;
    } u;
    T row[2 * TB];             /* published pivot row (double-buffered) */
    T col[2 * TB];             /* published pivot column (double-buffered) */
    T yrow[2 * 8];             /* published solution row in the sweeps */
    int ticket;
};

/* ----------------------------------------------------- register tiles --- */

/* Load an nr x nc corner of a 64x64 tile at G (pitch ldg); the rest is zero,
 * or the identity when pad_identity (keeps a padded diagonal tile regular). */
template <typename T>
__device__ __forceinline__ void rt_load(T (&a)[4][4], const T *__restrict__ G, int64_t ldg, int nr,
                                        int nc, bool pad_identity)
{
    const int tr = threadIdx.x >> 4, tc = threadIdx.x & 15;
#pragma unroll
    for (int qr = 0; qr < 4; ++qr) {
        const int i = trow(tr, qr);
#pragma unroll
        for (int qc = 0; qc < 4; ++qc) {
            const int j = trow(tc, qc);
            T v = (pad_identity && i == j) ? T(1) : T(0);
            if (i < nr && j < nc)
                v = G[(int64_t)i * ldg + j];
            a[qr][qc] = v;
        }
    }
}

template <typename T>
__device__ __forceinline__ void rt_store(const T (&a)[4][4], T *__restrict__ G, int64_t ldg, int nr,
                                         int nc)
{
    const int tr = threadIdx.x >> 4, tc = threadIdx.x & 15;
#pragma unroll
    for (int qr = 0; qr < 4; ++qr) {
        const int i = trow(tr, qr);
#pragma unroll
        for (int qc = 0; qc < 4; ++qc) {
            const int j = trow(tc, qc);
            if (i < nr && j < nc)
                G[(int64_t)i * ldg + j] = a[qr][qc];
        }
    }
}

template <typename T>
__device__ __forceinline__ void rt_store_lds(const T (&a)[4][4], T *S)
{
    const int tr = threadIdx.x >> 4, tc = threadIdx.x & 15;
#pragma unroll
    for (int qr = 0; qr < 4; ++qr)
#pragma unroll
        for (int qc = 0; qc < 4; ++qc)
            S[trow(tr, qr) * LDT + trow(tc, qc)] = a[qr][qc];
}

/*
 * In-register Doolittle LU of the leading nvalid x nvalid block of a 64x64
 * tile (Eq. 6-a: multipliers = column / pivot; Eq. 6-c: rank-1 update of the
 * active block).  Returns 0 or k+1 for the first exactly-zero pivot
 * (identical in every thread).
 */
template <typename T>
__device__ int rt_lu(T (&a)[4][4], T *s_row, T *s_col, int nvalid)
{
    const int tr = threadIdx.x >> 4, tc = threadIdx.x & 15;
    int zero_at = 0;
    for (int k = 0; k < nvalid; ++k) {
        T *rb = s_row + (k & 1) * TB;
        T *cb = s_col + (k & 1) * TB;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (trow(tr, q) == k) {
#pragma unroll
                for (int qc = 0; qc < 4; ++qc)
                    rb[trow(tc, qc)] = a[q][qc];
            }
            if (trow(tc, q) == k) {
#pragma unroll
                for (int qr = 0; qr < 4; ++qr)
                    cb[trow(tr, qr)] = a[qr][q];
            }
        }
        __syncthreads();
        const T p = rb[k];
        if (p == T(0) && zero_at == 0)
            zero_at = k + 1;
        const T rinv = T(1) / p;
        T u[4];
#pragma unroll
        for (int qc = 0; qc < 4; ++qc)
            u[qc] = rb[trow(tc, qc)];
#pragma unroll
        for (int qr = 0; qr < 4; ++qr) {
            const int i = trow(tr, qr);
            if (i > k) {
                const T l = cb[i] * rinv;
#pragma unroll
                for (int qc = 0; qc < 4; ++qc) {
                    const int j = trow(tc, qc);
                    if (j > k)
                        a[qr][qc] -= l * u[qc];
                    else if (j == k)
                        a[qr][qc] = l;
                }
            }
        }
    }
    __syncthreads();
    return zero_at;
}

/*
 * X <- L^{-1} X for a register tile X, L unit lower triangular in LDS
 * (pitch LDT): the U blocks right of a factored diagonal tile.
 */
template <typename T>
__device__ void rt_trsm_lower_unit(T (&x)[4][4], const T *sL, T *s_row, int nvalid)
{
    const int tr = threadIdx.x >> 4, tc = threadIdx.x & 15;
    for (int m = 0; m + 1 < nvalid; ++m) {
        T *rb = s_row + (m & 1) * TB;
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (trow(tr, q) == m) {
#pragma unroll
                for (int qc = 0; qc < 4; ++qc)
                    rb[trow(tc, qc)] = x[q][qc];
            }
        __syncthreads();
        T u[4];
#pragma unroll
        for (int qc = 0; qc < 4; ++qc)
            u[qc] = rb[trow(tc, qc)];
#pragma unroll
        for (int qr = 0; qr < 4; ++qr) {
            const int i = trow(tr, qr);
            if (i > m) {
                const T l = sL[i * LDT + m];
#pragma unroll
                for (int qc = 0; qc < 4; ++qc)
                    x[qr][qc] -= l * u[qc];
            }
        }
    }
    __syncthreads();
}

/*
 * X <- X U^{-1} for a register tile X, U upper triangular in LDS with the
 * reciprocals of its diagonal in s_rinv: the L blocks below a factored
 * diagonal tile.
 */
template <typename T>
__device__ void rt_trsm_upper_right(T (&x)[4][4], const T *sU, const T *s_rinv, T *s_col, int nvalid)
{
    const int tr = threadIdx.x >> 4, tc = threadIdx.x & 15;
    for (int m = 0; m < nvalid; ++m) {
        T *cb = s_col + (m & 1) * TB;
        const T r = s_rinv[m];
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (trow(tc, q) == m) {
#pragma unroll
                for (int qr = 0; qr < 4; ++qr) {
                    x[qr][q] *= r;
                    cb[trow(tr, qr)] = x[qr][q];
                }
            }
        __syncthreads();
        T l[4];
#pragma unroll
        for (int qr = 0; qr < 4; ++qr)
            l[qr] = cb[trow(tr, qr)];
#pragma unroll
        for (int qc = 0; qc < 4; ++qc) {
            const int j = trow(tc, qc);
            if (j > m) {
                const T u = sU[m * LDT + j];
#pragma unroll
                for (int qr = 0; qr < 4; ++qr)
                    x[qr][qc] -= l[qr] * u;
            }
        }
    }
    __syncthreads();
}

/* ------------------------------------------------------------ staging --- */

/* Copy an nr x nc corner of the 64x64 tile at G into LDS (pitch LDT), zero
 * elsewhere; TRANS stores element (r, c) at S[c*LDT + r]. */
template <typename T, bool TRANS>
__device__ __forceinline__ void stage64(T *S, const T *__restrict__ G, int64_t ldg, int nr, int nc)
{
    for (int idx = threadIdx.x; idx < TB * TB; idx += NT) {
        const int r = idx >> 6, c = idx & 63;
        const T v = (r < nr && c < nc) ? G[(int64_t)r * ldg + c] : T(0);
        if (TRANS)
            S[c * LDT + r] = v;
        else
            S[r * LDT + c] = v;
    }
}

/* Dense C addressing for wg_gemm64: element (r, c) of an nr x nc tile. */
template <typename T> struct DenseC {
    T *C;
    int64_t ldc;
    int nr, nc;
    __device__ __forceinline__ T *operator()(int r, int c) const
    {
        return (r < nr && c < nc) ? C + (int64_t)r * ldc + c : nullptr;
    }
};

/*
 * C(64x64 tile) -= A * B with A^T and B staged in LDS (pitch LDT, K = 64,
 * zero-padded): the trailing rank-64 update of Eq. 6-c applied 64 elimination
 * steps at a time, on the matrix cores.  `cref(r, c)` returns the address of
 * C's element (r, c), or nullptr for elements outside the tile's valid part.
 * Wave w computes the 32x32 quadrant (w / 2, w % 2).
 */
template <typename T, typename CRef>
__device__ void wg_gemm64(const CRef &cref, const T *sAT, const T *sB)
{
    typedef typename vec4<T>::type V;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
    const int lr = l & 15, lk = l >> 4;
    V acc[2][2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const T *p = cref(wm + 16 * bi + acc_row<T>(lk, r), wn + 16 * bj + lr);
                acc[bi][bj][r] = p ? *p : T(0);
            }
#pragma unroll 4
    for (int k = 0; k < TB; k += 4) {
        T a[2], b[2];
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
            a[bi] = -sAT[(k + lk) * LDT + wm + 16 * bi + lr];
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
            b[bj] = sB[(k + lk) * LDT + wn + 16 * bj + lr];
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj)
                acc[bi][bj] = mfma16(a[bi], b[bj], acc[bi][bj]);
    }
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                T *p = cref(wm + 16 * bi + acc_row<T>(lk, r), wn + 16 * bj + lr);
                if (p)
                    *p = acc[bi][bj][r];
            }
}

/* ------------------------------------------------ workgroup-level LU --- */

/*
 * Blocked right-looking Doolittle LU of one n x n matrix by one workgroup:
 * per 64-wide block step, factor the diagonal tile in registers, solve the U
 * blocks to its right and the L blocks below it, then apply the rank-64
 * update to the trailing tiles on the matrix cores.  Returns the first zero
 * pivot (1-based) or 0.
 */
template <typename T>
__device__ int wg_lu(T *__restrict__ A, int64_t lda, int n, TileSmem<T> &sm)
{
    const int nt = (n + TB - 1) / TB;
    int zero_at = 0;
    for (int kb = 0; kb < nt; ++kb) {
        const int k0 = kb * TB, kw = min(TB, n - k0);
        T *Akk = A + (int64_t)k0 * lda + k0;
        T a[4][4];
        rt_load(a, Akk, lda, kw, kw, true);
        const int z = rt_lu(a, sm.row, sm.col, kw);
        if (z && !zero_at)
            zero_at = k0 + z;
        rt_store(a, Akk, lda, kw, kw);
        if (kb + 1 == nt)
            break;
        rt_store_lds(a, sm.u.d.D);
        __syncthreads();
        if (threadIdx.x < TB)
            sm.u.d.rinv[threadIdx.x] = T(1) / sm.u.d.D[threadIdx.x * LDT + threadIdx.x];
        __syncthreads();
        for (int jb = kb + 1; jb < nt; ++jb) {
            const int j0 = jb * TB, jw = min(TB, n - j0);
            T *G = A + (int64_t)k0 * lda + j0;
            rt_load(a, G, lda, TB, jw, false);
            rt_trsm_lower_unit(a, sm.u.d.D, sm.row, TB);
            rt_store(a, G, lda, TB, jw);
        }
        for (int ib = kb + 1; ib < nt; ++ib) {
            const int i0 = ib * TB, iw = min(TB, n - i0);
            T *G = A + (int64_t)i0 * lda + k0;
            rt_load(a, G, lda, iw, TB, false);
            rt_trsm_upper_right(a, sm.u.d.D, sm.u.d.rinv, sm.col, TB);
            rt_store(a, G, lda, iw, TB);
        }
        __syncthreads();
        for (int ib = kb + 1; ib < nt; ++ib) {
            const int i0 = ib * TB, iw = min(TB, n - i0);
            stage64<T, true>(sm.u.g.AT, A + (int64_t)i0 * lda + k0, lda, iw, TB);
            for (int jb = kb + 1; jb < nt; ++jb) {
                const int j0 = jb * TB, jw = min(TB, n - j0);
                stage64<T, false>(sm.u.g.B, A + (int64_t)k0 * lda + j0, lda, TB, jw);
                __syncthreads();
                wg_gemm64(DenseC<T>{A + (int64_t)i0 * lda + j0, lda, iw, jw}, sm.u.g.AT, sm.u.g.B);
                __syncthreads();
            }
        }
    }
    __syncthreads();
    return zero_at;
}

/* ------------------------------------------------- triangular solves --- */

enum TriMode { TRI_L = 0, TRI_U = 1, TRI_UT = 2, TRI_LT = 3 };

/* Which triangle of the packed factor a mode reads, and whether it is read
 * transposed:  TRI_L  L (unit lower)   -> forward
 *              TRI_U  U (upper)        -> backward
 *              TRI_UT U^T (lower)      -> forward
 *              TRI_LT L^T (unit upper) -> backward */
__host__ __device__ constexpr bool tri_forward(int mode) { return mode == TRI_L || mode == TRI_UT; }
__host__ __device__ constexpr bool tri_trans(int mode) { return mode == TRI_UT || mode == TRI_LT; }
__host__ __device__ constexpr bool tri_unit(int mode) { return mode == TRI_L || mode == TRI_LT; }

/* Stages block (bi, bj) of the operator op(T) of `MODE` from the packed dense
 * factor into S (element (r, c) at S[r*LDT + c]), zero outside the matrix. */
template <typename T, int MODE> struct DenseOp {
    const T *LU;
    int64_t lda;
    int n;
    __device__ __forceinline__ void operator()(T *S, int bi, int bj) const
    {
        const int r0 = bi * TB, c0 = bj * TB;
        const int nr = min(TB, n - r0), nc = min(TB, n - c0);
        if (tri_trans(MODE)) /* op(r, c) = LU[c0 + c][r0 + r] */
            stage64<T, true>(S, LU + (int64_t)c0 * lda + r0, lda, nc, nr);
        else
            stage64<T, false>(S, LU + (int64_t)r0 * lda + c0, lda, nr, nc);
    }
};

/* Flag wait used by the multi-workgroup solves: thread 0 spins (bounded) on
 * flag == 1, then every thread performs an agent-scope acquire so its later
 * loads observe the producer's data. */
__device__ __forceinline__ void wait_flag(const int *flag, int *status)
{
    if (threadIdx.x == 0) {
        long spins = 0;
        while (__hip_atomic_load(flag, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == 0) {
            __builtin_amdgcn_s_sleep(2);
            if (++spins > (1L << 23)) {
                atomicOr(status, 1);
                break;
            }
        }
    }
    __syncthreads();
    __atomic_thread_fence(__ATOMIC_ACQUIRE);
}

/*
 * Solve one 64-row block `blk` of op(T) Y = B (Eq. 1's forward or backward
 * substitution, blocked): accumulate the contributions of the blocks solved
 * before it (at most `maxdep` of them, the earliest solved first), then sweep the
 * diagonal block.  NR <= 8 columns of B are handled (nrhs_here of them
 * valid).  With flags != nullptr the solved blocks come from other
 * workgroups and are waited for.  `op(S, bi, bj)` stages operator blocks.
 *
 * Thread t handles row rr = t / 4; for the off-diagonal products its quarter
 * q = t % 4 covers 16 of the 64 columns and the four partial sums are joined
 * with wavefront shuffles.
 */
template <typename T, int MODE, int NR, typename Op>
__device__ void solve_block(const Op &op, int n, T *__restrict__ B, int64_t ldb, int nrhs_here, int blk,
                            int maxdep, TileSmem<T> &sm, const int *flags, int *status)
{
    constexpr bool FWD = tri_forward(MODE);
    const int nb = (n + TB - 1) / TB;
    const int r0 = blk * TB, nr = min(TB, n - r0);
    const int t = threadIdx.x, rr = t >> 2, q = t & 3;
    T acc[NR];
#pragma unroll
    for (int c = 0; c < NR; ++c)
        acc[c] = T(0);
    const int ndep = min(maxdep, FWD ? blk : nb - 1 - blk);
    for (int d = 0; d < ndep; ++d) {
        const int j = FWD ? blk - ndep + d : blk + ndep - d;
        const int jw = min(TB, n - j * TB);
        op(sm.u.s.M, blk, j);
        if (flags)
            wait_flag(flags + j, status);
        for (int idx = t; idx < TB * NR; idx += NT) {
            const int r = idx / NR, c = idx % NR;
            sm.u.s.Y[r * NR + c] = (r < jw && c < nrhs_here) ? B[(int64_t)(j * TB + r) * ldb + c] : T(0);
        }
        __syncthreads();
#pragma unroll 4
        for (int cc = 0; cc < 16; ++cc) {
            const int col = 16 * q + cc;
            const T m = sm.u.s.M[rr * LDT + col];
#pragma unroll
            for (int c = 0; c < NR; ++c)
                acc[c] += m * sm.u.s.Y[col * NR + c];
        }
        __syncthreads();
    }
#pragma unroll
    for (int c = 0; c < NR; ++c) {
        acc[c] += __shfl_xor(acc[c], 1);
        acc[c] += __shfl_xor(acc[c], 2);
    }
    /* right-hand side of the diagonal block; thread (rr, q) keeps columns q, q+4 */
    constexpr int NC = (NR + 3) / 4;
    T y[NC];
#pragma unroll
    for (int h = 0; h < NC; ++h) {
        const int c = q + 4 * h;
        T v = T(0);
#pragma unroll
        for (int cc = 0; cc < NR; ++cc)
            if (cc == c)
                v = acc[cc];
        y[h] = (rr < nr && c < nrhs_here) ? B[(int64_t)(r0 + rr) * ldb + c] - v : T(0);
    }
    op(sm.u.s.M, blk, blk);
    __syncthreads();
    for (int s = 0; s < nr; ++s) {
        const int m = FWD ? s : nr - 1 - s;
        T *yb = sm.yrow + (s & 1) * 8;
        if (rr == m) {
#pragma unroll
            for (int h = 0; h < NC; ++h) {
                if (!tri_unit(MODE))
                    y[h] = y[h] / sm.u.s.M[m * LDT + m];
                yb[q + 4 * h] = y[h];
            }
        }
        __syncthreads();
        const bool after = FWD ? (rr > m) : (rr < m);
        if (after && rr < nr) {
            const T coef = sm.u.s.M[rr * LDT + m];
#pragma unroll
            for (int h = 0; h < NC; ++h)
                y[h] -= coef * yb[q + 4 * h];
        }
    }
#pragma unroll
    for (int h = 0; h < NC; ++h) {
        const int c = q + 4 * h;
        if (rr < nr && c < nrhs_here)
            B[(int64_t)(r0 + rr) * ldb + c] = y[h];
    }
    __syncthreads();
}

/* Whole triangular solve of op(T) by one workgroup, block after block. */
template <typename T, int MODE, int NR>
__device__ void wg_solve(const T *LU, int64_t lda, int n, T *B, int64_t ldb, int nrhs_here, TileSmem<T> &sm)
{
    const int nb = (n + TB - 1) / TB;
    const DenseOp<T, MODE> op{LU, lda, n};
    for (int s = 0; s < nb; ++s) {
        const int blk = tri_forward(MODE) ? s : nb - 1 - s;
        solve_block<T, MODE, NR>(op, n, B, ldb, nrhs_here, blk, nb, sm, nullptr, nullptr);
    }
}

} /* namespace ebv */

#endif /* EBV_DEVICE_HPP */
