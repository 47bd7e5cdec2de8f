/*
 * Device building blocks for the EbV LU kernels (gfx950, wave64).
 *
 * Elimination (Eq. 6-a, 6-c) is blocked in 64 x 64 tiles.  The sequential
 * part of a block step -- the 64 pivot steps of the diagonal tile and the
 * triangular solves of the U/L blocks next to it -- runs in single waves that
 * keep the tile in registers, one row or column per lane, and pass the pivot
 * step's values between lanes with readlane broadcasts: no barrier and no LDS
 * round trip per pivot step.  The rank-64 trailing update, where the flops
 * are, runs on the FP64 (or FP32) matrix cores.  LDS stages the factored
 * diagonal tile (the paper's use of shared memory) and the matrix-core
 * operands.
 *
 * The EbV equal-work pairing (paper: join the longest vector with the
 * shortest) is applied where parallel units receive unequal work: whole
 * systems of a ragged batch are taken largest-with-smallest (ebv_pairing.h).
 */
#ifndef EBV_DEVICE_HPP
#define EBV_DEVICE_HPP

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

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

/* Reciprocal: hardware estimate refined by Newton steps (each squares the
 * relative error), within an ulp or two of 1/x; exact zeros give inf. */
__device__ __forceinline__ double recip(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-x, r, 1.0);
    return __builtin_fma(r, e, r);
}
__device__ __forceinline__ float recip(float x)
{
    float r = __builtin_amdgcn_rcpf(x);
    const float e = __builtin_fmaf(-x, r, 1.0f);
    return __builtin_fmaf(r, e, r);
}

/* Wave-wide broadcast of lane `lane`'s value (lane uniform). */
__device__ __forceinline__ double bcast(double v, int lane)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ float bcast(float v, int lane)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

/* -------------------------------------------------------- LDS layouts --- */

/* Scratch shared by the tile routines of one workgroup. */
template <typename T> struct TileSmem {
    T t0[TB * LDT];   /* factored diagonal tile / A^T operand / operator tile */
    T t1[TB * LDT];   /* sweep output tile / B operand / staged solved block */
    T rinv[TB];       /* reciprocals of the diagonal of t0 */
    T row[2 * TB];    /* published pivot row (double-buffered) */
    T col[2 * TB];    /* published pivot column (double-buffered) */
    int ticket;
    int zflag;        /* zero-pivot report shared by the workgroup */
};

/* Store the nr x nc corner of an LDS tile (pitch LDT) to G (pitch ldg). */
template <typename T>
__device__ __forceinline__ void lds_store_tile(const T *S, T *__restrict__ G, int64_t ldg, int nr, int nc)
{
    for (int idx = threadIdx.x; idx < TB * TB; idx += NT) {
        const int r = idx >> 6, c = idx & 63;
        if (r < nr && c < nc)
            G[(int64_t)r * ldg + c] = S[r * LDT + c];
    }
}

/* ------------------------------------------- register-tile sweeps --- */

/*
 * A 64 x 64 tile held by the whole workgroup, 16 values per thread: thread
 * t = 16*tr + tc owns rows ebv_row(tr, q) and columns ebv_row(tc, q),
 * q = 0..3 -- the EbV-joined pairs {v, 63-v} (ebv_pairing.h), so each
 * thread's share of every elimination step is within one row of the mean.
 * A step publishes the pivot row and column through LDS (double-buffered,
 * one barrier per step).  The register slot that holds row or column k is
 * constant over each quarter of k (rows 0-15 slot 0, 16-31 slot 2, 32-47
 * slot 3, 48-63 slot 1), so the sweeps run four phases with the slot as a
 * compile-time constant and no register array is indexed at run time.
 */
__device__ __forceinline__ int trow(int u, int q) { return ebv_row(u, q, 16, TB); }

template <typename F> __device__ __forceinline__ void four_phases(F &&step)
{
#pragma unroll 1
    for (int k = 0; k < 16; ++k)
        step(k, k, std::integral_constant<int, 0>());
#pragma unroll 1
    for (int k = 16; k < 32; ++k)
        step(k, k - 16, std::integral_constant<int, 2>());
#pragma unroll 1
    for (int k = 32; k < 48; ++k)
        step(k, 47 - k, std::integral_constant<int, 3>());
#pragma unroll 1
    for (int k = 48; k < 64; ++k)
        step(k, 63 - k, std::integral_constant<int, 1>());
}

/* Load the nr x nc corner of the 64x64 tile at G into the register tile;
 * the rest is zero, or the identity when pad_identity. */
template <typename T>
__device__ __forceinline__ void rt_load(T (&a)[4][4], const T *__restrict__ G, int64_t ldg, int nr, int nc,
                                        bool pad_identity)
{
    const int tr = threadIdx.x >> 4, tc = threadIdx.x & 15;
#pragma unroll
    for (int qr = 0; qr < 4; ++qr) {
        const int i = trow(tr, qr);
#pragma unroll
        for (int qc = 0; qc < 4; ++qc) {
            const int j = trow(tc, qc);
            a[qr][qc] = (i < nr && j < nc) ? G[(int64_t)i * ldg + j] : ((pad_identity && i == j) ? T(1) : T(0));
        }
    }
}
template <typename T>
__device__ __forceinline__ void rt_store(const T (&a)[4][4], T *__restrict__ G, int64_t ldg, int nr, int nc)
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
 * Doolittle LU of a register tile (Eq. 6-a: multipliers = column / pivot;
 * Eq. 6-c: rank-1 update of the active block).  The tile is left factored
 * in the registers (strict lower part L, upper part U) and 1/U_kk in
 * sm.rinv.  A tile padded with the identity beyond nvalid is swept to the
 * end, which keeps the identity there.  Returns 0 or k+1 for the first
 * exactly-zero pivot among the first nvalid (same in every thread).
 */
template <typename T>
__device__ int rt_lu(T (&a)[4][4], TileSmem<T> &sm, int nvalid)
{
    const int t = threadIdx.x, tr = t >> 4, tc = t & 15;
    int ri[4], cj[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        ri[q] = trow(tr, q);
        cj[q] = trow(tc, q);
    }
    int zero_at = 0;
    four_phases([&](int k, int ou, auto osc) {
        constexpr int os = decltype(osc)::value;
        T *rb = sm.row + (k & 1) * TB;
        T *cb = sm.col + (k & 1) * TB;
        if (tr == ou) {
#pragma unroll
            for (int qc = 0; qc < 4; ++qc)
                rb[cj[qc]] = a[os][qc];
        }
        if (tc == ou) {
#pragma unroll
            for (int qr = 0; qr < 4; ++qr)
                cb[ri[qr]] = a[qr][os];
        }
        __syncthreads();
        const T p = rb[k];
        T u[4], lv[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            u[q] = rb[cj[q]];
            lv[q] = cb[ri[q]];
        }
        if (p == T(0) && zero_at == 0 && k < nvalid)
            zero_at = k + 1;
        const T rinv = recip(p);
        if (t == 0)
            sm.rinv[k] = rinv;
        T um[4];
#pragma unroll
        for (int qc = 0; qc < 4; ++qc)
            um[qc] = cj[qc] > k ? u[qc] : T(0);
        const bool colk = tc == ou;
#pragma unroll
        for (int qr = 0; qr < 4; ++qr) {
            const T l = lv[qr] * rinv;
            const bool below = ri[qr] > k;
            const T lm = below ? l : T(0);
            a[qr][os] = (colk && below) ? l : a[qr][os];
#pragma unroll
            for (int qc = 0; qc < 4; ++qc)
                a[qr][qc] = __builtin_fma(-lm, um[qc], a[qr][qc]);
        }
    });
    __syncthreads();
    return zero_at;
}

/* X <- L^{-1} X for a register tile X, L the unit lower part of the factored
 * tile in LDS (pitch LDT): the U blocks right of a diagonal tile. */
template <typename T>
__device__ void rt_trsm_lower_unit(T (&x)[4][4], const T *L, TileSmem<T> &sm)
{
    const int tr = threadIdx.x >> 4, tc = threadIdx.x & 15;
    int ri[4], cj[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        ri[q] = trow(tr, q);
        cj[q] = trow(tc, q);
    }
    four_phases([&](int m, int ou, auto osc) {
        constexpr int os = decltype(osc)::value;
        T *rb = sm.row + (m & 1) * TB;
        T lm[4];
#pragma unroll
        for (int qr = 0; qr < 4; ++qr)
            lm[qr] = ri[qr] > m ? L[ri[qr] * LDT + m] : T(0);
        if (tr == ou) {
#pragma unroll
            for (int qc = 0; qc < 4; ++qc)
                rb[cj[qc]] = x[os][qc];
        }
        __syncthreads();
        T u[4];
#pragma unroll
        for (int qc = 0; qc < 4; ++qc)
            u[qc] = rb[cj[qc]];
#pragma unroll
        for (int qr = 0; qr < 4; ++qr)
#pragma unroll
            for (int qc = 0; qc < 4; ++qc)
                x[qr][qc] = __builtin_fma(-lm[qr], u[qc], x[qr][qc]);
    });
    __syncthreads();
}

/* X <- X U^{-1} for a register tile X, U the upper part of the factored tile
 * in LDS with 1/U_mm in rinv: the L blocks below a diagonal tile. */
template <typename T>
__device__ void rt_trsm_upper_right(T (&x)[4][4], const T *U, const T *rinv, TileSmem<T> &sm)
{
    const int tr = threadIdx.x >> 4, tc = threadIdx.x & 15;
    int ri[4], cj[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        ri[q] = trow(tr, q);
        cj[q] = trow(tc, q);
    }
    four_phases([&](int m, int ou, auto osc) {
        constexpr int os = decltype(osc)::value;
        T *cb = sm.col + (m & 1) * TB;
        T um[4];
#pragma unroll
        for (int qc = 0; qc < 4; ++qc)
            um[qc] = cj[qc] > m ? U[m * LDT + cj[qc]] : T(0);
        if (tc == ou) {
            const T r = rinv[m];
#pragma unroll
            for (int qr = 0; qr < 4; ++qr) {
                x[qr][os] *= r;
                cb[ri[qr]] = x[qr][os];
            }
        }
        __syncthreads();
        T l[4];
#pragma unroll
        for (int qr = 0; qr < 4; ++qr)
            l[qr] = cb[ri[qr]];
#pragma unroll
        for (int qr = 0; qr < 4; ++qr)
#pragma unroll
            for (int qc = 0; qc < 4; ++qc)
                x[qr][qc] = __builtin_fma(-l[qr], um[qc], x[qr][qc]);
    });
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
 * blocks to its right and the L blocks below it against it (kept in LDS),
 * then apply the rank-64 update to the trailing tiles on the matrix cores.
 * Returns the first zero pivot (1-based) or 0.
 */
template <typename T>
__device__ __forceinline__ int wg_lu(T *__restrict__ A, int64_t lda, int n, TileSmem<T> &sm)
{
    const int nt = (n + TB - 1) / TB;
    int zero_at = 0;
    for (int kb = 0; kb < nt; ++kb) {
        const int k0 = kb * TB, kw = min(TB, n - k0);
        T *Akk = A + (int64_t)k0 * lda + k0;
        T a[4][4];
        rt_load(a, Akk, lda, kw, kw, true);
        const int z = rt_lu(a, sm, kw);
        if (z && !zero_at)
            zero_at = k0 + z;
        rt_store(a, Akk, lda, kw, kw);
        if (kb + 1 == nt)
            break;
        rt_store_lds(a, sm.t0);
        __syncthreads();
        for (int jb = kb + 1; jb < nt; ++jb) {
            const int j0 = jb * TB, jw = min(TB, n - j0);
            T *G = A + (int64_t)k0 * lda + j0;
            rt_load(a, G, lda, TB, jw, false);
            rt_trsm_lower_unit(a, sm.t0, sm);
            rt_store(a, G, lda, TB, jw);
        }
        for (int ib = kb + 1; ib < nt; ++ib) {
            const int i0 = ib * TB, iw = min(TB, n - i0);
            T *G = A + (int64_t)i0 * lda + k0;
            rt_load(a, G, lda, iw, TB, false);
            rt_trsm_upper_right(a, sm.t0, sm.rinv, sm);
            rt_store(a, G, lda, iw, TB);
        }
        __syncthreads();
        for (int ib = kb + 1; ib < nt; ++ib) {
            const int i0 = ib * TB, iw = min(TB, n - i0);
            stage64<T, true>(sm.t0, A + (int64_t)i0 * lda + k0, lda, iw, TB);
            for (int jb = kb + 1; jb < nt; ++jb) {
                const int j0 = jb * TB, jw = min(TB, n - j0);
                stage64<T, false>(sm.t1, A + (int64_t)k0 * lda + j0, lda, TB, jw);
                __syncthreads();
                wg_gemm64(DenseC<T>{A + (int64_t)i0 * lda + j0, lda, iw, jw}, sm.t0, sm.t1);
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
    /* Row rr, columns 16q..16q+15 of operator block (bi, bj), zero outside. */
    __device__ __forceinline__ void seg(int bi, int bj, int rr, int q, T (&m)[16]) const
    {
        const int r = bi * TB + rr, c0 = bj * TB + 16 * q;
#pragma unroll
        for (int cc = 0; cc < 16; ++cc) {
            const int c = c0 + cc;
            const bool ok = r < n && c < n;
            m[cc] = ok ? (tri_trans(MODE) ? LU[(int64_t)c * lda + r] : LU[(int64_t)r * lda + c]) : T(0);
        }
    }
};


/* Flag wait used by the multi-workgroup solves: thread 0 spins (bounded) on
 * flag == 1, then every thread performs an agent-scope acquire so its later
 * loads observe the producer's data. */
__device__ __forceinline__ void wait_flag(const int *flag, int *status)
{
    if (threadIdx.x == 0) {
        /* relaxed polls (no cache invalidation per poll), bounded */
        long spins = 0;
        while (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
            __builtin_amdgcn_s_sleep(1);
            if (++spins > (1L << 24)) {
                atomicOr(status, 1);
                break;
            }
        }
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

/*
 * Solve one 64-row block `blk` of op(T) Y = B (Eq. 1's forward or backward
 * substitution, blocked): accumulate the contributions of the blocks solved
 * before it (at most `maxdep` of them, the earliest solved first), then sweep
 * the diagonal block.  NR <= 8 columns of B are handled (nrhs_here of them
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
    T *Y = sm.t1;
    T mc[16], mn[16];
    if (ndep > 0)
        op.seg(blk, FWD ? blk - ndep : blk + ndep, rr, q, mc);
    for (int d = 0; d < ndep; ++d) {
        const int j = FWD ? blk - ndep + d : blk + ndep - d;
        const int jw = min(TB, n - j * TB);
        if (d + 1 < ndep)
            op.seg(blk, FWD ? j + 1 : j - 1, rr, q, mn);
        if (flags)
            wait_flag(flags + j, status);
        for (int idx = t; idx < TB * NR; idx += NT) {
            const int r = idx / NR, c = idx % NR;
            Y[r * NR + c] = (r < jw && c < nrhs_here) ? B[(int64_t)(j * TB + r) * ldb + c] : T(0);
        }
        __syncthreads();
#pragma unroll
        for (int cc = 0; cc < 16; ++cc) {
            const int col = 16 * q + cc;
#pragma unroll
            for (int c = 0; c < NR; ++c)
                acc[c] = __builtin_fma(mc[cc], Y[col * NR + c], acc[c]);
        }
        __syncthreads();
#pragma unroll
        for (int cc = 0; cc < 16; ++cc)
            mc[cc] = mn[cc];
    }
#pragma unroll
    for (int c = 0; c < NR; ++c) {
        acc[c] += __shfl_xor(acc[c], 1);
        acc[c] += __shfl_xor(acc[c], 2);
    }
    /* right-hand side of the diagonal block, row-major in LDS */
    if (q == 0)
#pragma unroll
        for (int c = 0; c < NR; ++c)
            Y[rr * NR + c] = (rr < nr && c < nrhs_here) ? B[(int64_t)(r0 + rr) * ldb + c] - acc[c] : T(0);
    op(sm.t0, blk, blk);
    __syncthreads();
    /* diagonal block: wave 0 sweeps it, lane r holding row r; the finished
     * row's values are broadcast with readlane, so no barrier is needed */
    if (t < TB) {
        const T *M = sm.t0;
        const int r = t;
        T y[NR];
#pragma unroll
        for (int c = 0; c < NR; ++c)
            y[c] = Y[r * NR + c];
        const T rin = (!tri_unit(MODE) && r < nr) ? recip(M[r * LDT + r]) : T(1);
        for (int s = 0; s < nr; ++s) {
            const int m = FWD ? s : nr - 1 - s;
            const bool after = FWD ? (r > m) : (r < m);
            const T cf = after ? M[r * LDT + m] : T(0);
#pragma unroll
            for (int c = 0; c < NR; ++c) {
                if (!tri_unit(MODE))
                    y[c] = (r == m) ? y[c] * rin : y[c];
                const T ym = bcast(y[c], m);
                y[c] = __builtin_fma(-cf, ym, y[c]);
            }
        }
        if (r < nr)
#pragma unroll
            for (int c = 0; c < NR; ++c)
                if (c < nrhs_here)
                    B[(int64_t)(r0 + r) * ldb + c] = y[c];
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
