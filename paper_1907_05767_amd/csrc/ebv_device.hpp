/*
 * Device building blocks for the EbV LU kernels (gfx950, wave64).
 *
 * Elimination (Eq. 6-a, 6-c) is blocked in 64 x 64 tiles.  A diagonal tile is
 * factored in LDS in four 16-column panels (tile_lu16): one wave runs the 16
 * pivot steps of a panel with one row per lane and the pivot row broadcast
 * by readlane, one wave solves the 16 U rows beside it, and the rank-16
 * update of the rest runs on the matrix cores.  The inverses of the tile's
 * two triangular factors follow by block recursion on the matrix cores
 * (tile_inv16), so that every triangular solve against a diagonal tile --
 * the U blocks right of it, the L blocks below it, the blocks of a
 * substitution -- becomes a 64 x 64 product.  The rank-64 trailing update,
 * where the flops are, runs on the FP64 (or FP32) matrix cores.
 *
 * The EbV equal-work pairing (join the longest unit of work with the
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

/* Index of the calling wave in its workgroup, as a wave-uniform (scalar)
 * value, so that branches on it are uniform branches. */
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

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

/* ---------------------------------------------- compiler controls --- */

/* Keeps the compiler (IR passes and the machine scheduler) from moving
 * loads across this point, which bounds the registers a fully unrolled
 * substitution would otherwise fill with preloaded coefficients; emits no
 * instruction. */
__device__ __forceinline__ void lds_fence_compiler()
{
    asm volatile("" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
}

/* Pins the 16 values of a substitution step: every update of them issued
 * before this point is complete here, and no load is moved across it, so a
 * fully unrolled substitution keeps only one step's coefficients live. */
template <typename T> __device__ __forceinline__ void pin16(T (&x)[16])
{
    asm volatile(""
                 : "+v"(x[0]), "+v"(x[1]), "+v"(x[2]), "+v"(x[3]), "+v"(x[4]), "+v"(x[5]), "+v"(x[6]),
                   "+v"(x[7]), "+v"(x[8]), "+v"(x[9]), "+v"(x[10]), "+v"(x[11]), "+v"(x[12]), "+v"(x[13]),
                   "+v"(x[14]), "+v"(x[15])
                 :
                 : "memory");
    __builtin_amdgcn_sched_barrier(0);
}

/* Returns p unchanged, opaquely: address arithmetic based on the result
 * cannot be hoisted above this point (out of an enclosing loop), which keeps
 * the many LDS addresses of a fully unrolled tile routine from staying live
 * across the whole loop; emits no instruction. */
template <typename T> __device__ __forceinline__ T *launder(T *p)
{
    int off = 0;
    asm volatile("" : "+v"(off));
    return p + off;
}
template <typename T> __device__ __forceinline__ const T *launder(const T *p)
{
    int off = 0;
    asm volatile("" : "+v"(off));
    return p + off;
}
__device__ __forceinline__ int launder(int v)
{
    asm volatile("" : "+v"(v));
    return v;
}

/* -------------------------------------------------------- LDS layouts --- */

/* Scratch shared by the tile routines of one workgroup. */
template <typename T> struct TileSmem {
    T t0[TB * LDT];   /* diagonal tile / staged operand / operator tile */
    T t1[TB * LDT];   /* inverses of the factors / B operand / staged solved block */
    T rinv[TB];       /* reciprocals of the pivots of t0 */
    T aux[32 + 256];  /* tile_lu16 scratch */
    int ticket;
    int zflag;        /* zero-pivot report shared by the workgroup */
    int avail;        /* blocks known solved (multi-workgroup solves) */
};

/*
 * Element-wise pass over a 64 x 64 tile by the workgroup: thread t handles
 * column t % 64 and rows t / 64 + 4i, i = 0..15, and issues all 16 of its
 * loads before any of its stores, so that the memory latency is paid once
 * rather than once per element.  ld(r, c) returns element (r, c); st(r, c, v)
 * stores it.
 */
template <typename T, typename LD, typename ST> __device__ __forceinline__ void tile_xfer(LD &&ld, ST &&st)
{
    static_assert(NT == 4 * TB, "one column per lane, four rows per pass");
    const int c = launder((int)threadIdx.x & 63), r0 = launder((int)threadIdx.x >> 6);
    T v[16];
#pragma unroll
    for (int i = 0; i < 16; ++i)
        v[i] = ld(r0 + 4 * i, c);
#pragma unroll
    for (int i = 0; i < 16; ++i)
        st(r0 + 4 * i, c, v[i]);
}

/* Store the nr x nc corner of an LDS tile (pitch LDT) to G (pitch ldg). */
template <typename T>
__device__ __forceinline__ void lds_store_tile(const T *S, T *__restrict__ G, int64_t ldg, int nr, int nc)
{
    tile_xfer<T>([&](int r, int c) { return S[r * LDT + c]; },
                 [&](int r, int c, T v) {
                     if (r < nr && c < nc)
                         G[(int64_t)r * ldg + c] = v;
                 });
}

/* ------------------------------------------------------------ staging --- */

/* Copy an nr x nc corner of the 64x64 tile at G into LDS (pitch LDT), zero
 * elsewhere; TRANS stores element (r, c) at S[c*LDT + r]. */
template <typename T, bool TRANS>
__device__ __forceinline__ void stage64(T *S, const T *__restrict__ G, int64_t ldg, int nr, int nc)
{
    tile_xfer<T>([&](int r, int c) { return (r < nr && c < nc) ? G[(int64_t)r * ldg + c] : T(0); },
                 [&](int r, int c, T v) {
                     if (TRANS)
                         S[c * LDT + r] = v;
                     else
                         S[r * LDT + c] = v;
                 });
}

/* Two stage64 transfers (non-transposed) with all loads of both issued
 * before any store: one memory latency for the pair. */
template <typename T>
__device__ __forceinline__ void stage64x2(T *S1, const T *__restrict__ G1, int64_t ld1, int nr1, int nc1, T *S2,
                                          const T *__restrict__ G2, int64_t ld2, int nr2, int nc2)
{
    const int c = launder((int)threadIdx.x & 63), r0 = launder((int)threadIdx.x >> 6);
    T v1[16], v2[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int r = r0 + 4 * i;
        v1[i] = (r < nr1 && c < nc1) ? G1[(int64_t)r * ld1 + c] : T(0);
        v2[i] = (r < nr2 && c < nc2) ? G2[(int64_t)r * ld2 + c] : T(0);
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int r = r0 + 4 * i;
        S1[r * LDT + c] = v1[i];
        S2[r * LDT + c] = v2[i];
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
__device__ __forceinline__ void wg_gemm64(const CRef &cref, const T *sAT, const T *sB)
{
    typedef typename vec4<T>::type V;
    const int w = wave_id(), l = threadIdx.x & 63;
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

/* --------------------------------------------- blocked tile factor --- */


/* Accumulator of one 16x16 matrix-core block: element r of lane l is
 * (acc_row<T>(l / 16, r), l % 16). */
template <typename T>
__device__ __forceinline__ void acc_load(typename vec4<T>::type &acc, const T *C, int ldc)
{
    const int l = threadIdx.x & 63, lr = l & 15, lk = l >> 4;
#pragma unroll
    for (int r = 0; r < 4; ++r)
        acc[r] = C[acc_row<T>(lk, r) * ldc + lr];
}
template <typename T>
__device__ __forceinline__ void acc_store(const typename vec4<T>::type &acc, T *C, int ldc)
{
    const int l = threadIdx.x & 63, lr = l & 15, lk = l >> 4;
#pragma unroll
    for (int r = 0; r < 4; ++r)
        C[acc_row<T>(lk, r) * ldc + lr] = acc[r];
}

/* One wave: acc += A(16 x K) * B(K x 16) with fa(r, k) = A[r][k] and
 * fb(k, c) = B[k][c].  Inside each group of four, lane group lk contributes
 * k index acc_row<T>(lk, ks): the order in which an accumulator holds its
 * rows, so an accumulator can serve directly as the B operand of the next
 * product (see wave_mma16_acc). */
template <typename T, int K, typename FA, typename FB>
__device__ __forceinline__ void wave_mma16(typename vec4<T>::type &acc, FA &&fa, FB &&fb)
{
    const int l = threadIdx.x & 63, lr = l & 15, lk = l >> 4;
#pragma unroll
    for (int k0 = 0; k0 < K; k0 += 16)
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const int k = k0 + acc_row<T>(lk, ks);
            acc = mfma16(fa(lr, k), fb(k, lr), acc);
        }
}
/* One wave: acc += A(16 x 16) * Bacc with the B operand an accumulator. */
template <typename T, typename FA>
__device__ __forceinline__ void wave_mma16_acc(typename vec4<T>::type &acc, FA &&fa,
                                               const typename vec4<T>::type &b)
{
    const int l = threadIdx.x & 63, lr = l & 15, lk = l >> 4;
#pragma unroll
    for (int ks = 0; ks < 4; ++ks)
        acc = mfma16(fa(lr, acc_row<T>(lk, ks)), b[ks], acc);
}

/*
 * Doolittle LU (Eq. 6-a, 6-c) of the 64 x 64 tile S in LDS (pitch LDT), in
 * place, blocked in four 16-column panels.  Per panel, wave 0 alone:
 *   - factors the panel: 16 pivot steps, two at a time, with one row per
 *     lane and the panel's 16 columns in registers; the two pivot rows' lanes
 *     write them to LDS and every lane reads them back as a broadcast (a
 *     wave's LDS accesses complete in order, so no barrier is involved);
 *   - solves the 16 U rows to the panel's right against the panel's
 *     unit-lower block (one column per lane), reading the L coefficients as
 *     broadcasts from a transposed copy in LDS;
 * then all waves apply the rank-16 update to the rest on the matrix cores.
 * aux: 32 + 16*16 elements of LDS scratch.  rinv receives 1/U_kk.  Rows and
 * columns past nvalid must hold the identity, which the sweep keeps.
 * Returns 0 or k+1 for the first exactly-zero pivot k < nvalid (the same in
 * every thread).  While wave 0 factors panel p >= 1, waves 1..3 call
 * done(p - 1, 0): panel p - 1 (its columns below the diagonal, its rows right
 * of the diagonal, its diagonal block and rinv) is final then and no longer
 * touched, so a caller can start publishing it; from p >= 2 they first call
 * done(p - 2, 1), where a caller can wait for the previous panel's stores
 * (a panel later, so that no barrier of the factorization waits for memory;
 * done(2, 1) is left to the caller, after the factorization).
 */
struct NoPanelHook {
    __device__ __forceinline__ void operator()(int, int) const {}
};
template <typename T, typename Done = NoPanelHook>
__device__ __forceinline__ int tile_lu16(T *S, T *rinv, T *aux, int nvalid, int *zflag, Done &&done = Done())
{
    typedef typename vec4<T>::type V;
    S = launder(S);
    rinv = launder(rinv);
    T *R = launder(aux), *LT = R + 32; /* two pivot rows; L11 transposed (pitch 16) */
    const int t = threadIdx.x, w = wave_id(), l = launder(t & 63);
    int zero_at = 0;
#pragma unroll 1
    for (int p = 0; p < 4; ++p) {
        const int c0 = 16 * p;
        if (w == 0) {
            T v[16];
#pragma unroll
            for (int j = 0; j < 16; ++j)
                v[j] = S[l * LDT + c0 + j];
            /* pivots in pairs (a, a+1): both pivot rows travel in one LDS
             * round trip, and the two rank-1 updates are applied as one
             * rank-2 update from the rows as read: with m = u1[a] / u0[a]
             * and the second pivot row u1 - m u0,
             *   v -= l0 u0 + l1 (u1 - m u0) = (l0 - l1 m) u0 + l1 u1,
             * which also brings row a+1 itself up to date (its l1 is 0). */
#pragma unroll
            for (int a = 0; a < 16; a += 2) {
                const int pr = c0 + a;
                if (l == pr || l == pr + 1)
#pragma unroll
                    for (int j = a; j < 16; ++j)
                        R[(l - pr) * 16 + j] = v[j];
                __builtin_amdgcn_wave_barrier();
                T u0[16], u1[16];
#pragma unroll
                for (int j = a; j < 16; ++j) {
                    u0[j] = R[j];
                    u1[j] = R[16 + j];
                }
                const T p0 = u0[a];
                const T r0 = recip(p0);
                const T m10 = u1[a] * r0;
                const T p1 = __builtin_fma(-m10, u0[a + 1], u1[a + 1]);
                const T r1 = recip(p1);
                if (p0 == T(0) && zero_at == 0 && pr < nvalid)
                    zero_at = pr + 1;
                if (p1 == T(0) && zero_at == 0 && pr + 1 < nvalid)
                    zero_at = pr + 2;
                if (l == 0) {
                    rinv[pr] = r0;
                    rinv[pr + 1] = r1;
                }
                const T l0 = l > pr ? v[a] * r0 : T(0);
                const T x1 = __builtin_fma(-l0, u0[a + 1], v[a + 1]);
                const T l1 = l > pr + 1 ? x1 * r1 : T(0);
                const T c0f = __builtin_fma(-l1, m10, l0);
                v[a] = l > pr ? l0 : v[a];
                v[a + 1] = l > pr + 1 ? l1 : (l == pr + 1 ? x1 : v[a + 1]);
#pragma unroll
                for (int j = a + 2; j < 16; ++j)
                    v[j] = __builtin_fma(-c0f, u0[j], __builtin_fma(-l1, u1[j], v[j]));
                __builtin_amdgcn_wave_barrier();
            }
#pragma unroll
            for (int j = 0; j < 16; ++j)
                S[l * LDT + c0 + j] = v[j];
            if (p < 3) {
                /* U rows c0..c0+15 right of the panel: L11^{-1} A12, lane = column */
                if (l >= c0 && l < c0 + 16)
#pragma unroll
                    for (int kk = 0; kk < 16; ++kk)
                        LT[kk * 16 + (l - c0)] = v[kk];
                __builtin_amdgcn_wave_barrier();
                const bool act = l >= c0 + 16;
                T x[16];
#pragma unroll
                for (int i = 0; i < 16; ++i)
                    x[i] = S[(c0 + i) * LDT + l];
#pragma unroll
                for (int kk = 0; kk < 15; ++kk)
#pragma unroll
                    for (int i = kk + 1; i < 16; ++i)
                        x[i] = __builtin_fma(-LT[kk * 16 + i], x[kk], x[i]);
                if (act)
#pragma unroll
                    for (int i = 0; i < 16; ++i)
                        S[(c0 + i) * LDT + l] = x[i];
            }
        } else if (p > 0) {
            if (p > 1)
                done(p - 2, 1);
            done(p - 1, 0);
        }
        __syncthreads();
        if (p == 3)
            break;
        const int nb2 = 3 - p;
        for (int b = w; b < nb2 * nb2; b += 4) {
            const int i0 = c0 + 16 + 16 * (b / nb2), j0 = c0 + 16 + 16 * (b % nb2);
            V acc;
            acc_load<T>(acc, S + i0 * LDT + j0, LDT);
            wave_mma16<T, 16>(
                acc, [&](int r, int k) { return -S[(i0 + r) * LDT + c0 + k]; },
                [&](int k, int c) { return S[(c0 + k) * LDT + j0 + c]; });
            acc_store<T>(acc, S + i0 * LDT + j0, LDT);
        }
        __syncthreads();
    }
    if (t == 0)
        *zflag = zero_at;
    __syncthreads();
    return *zflag;
}

/* The 16 x 16 diagonal blocks of the inverses of the factors of a tile
 * factored by tile_lu16 (S, with 1/U_kk in rinv), by substitution against
 * the identity (wave 0 the four of L, wave 1 the four of U, one column per
 * lane), packed in P (LDS, pitch LDT) as tile_inv16 packs the whole
 * inverses: L_pp^{-1} in the strict lower part of diagonal block p (its unit
 * diagonal implied), U_pp^{-1} in its upper part.  The off-diagonal blocks
 * of P are left untouched. */
template <typename T>
__device__ __forceinline__ void tile_diag_inv16(const T *S, const T *rinv, T *P)
{
    S = launder(S);
    P = launder(P);
    rinv = launder(rinv);
    const int t = threadIdx.x, w = wave_id(), l = launder(t & 63), bp = l >> 4, c = l & 15;
    if (w == 0) {
        const T *L = S + 16 * bp * (LDT + 1);
        T x[16];
#pragma unroll
        for (int i = 0; i < 16; ++i)
            x[i] = (i == c) ? T(1) : T(0);
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
#pragma unroll
            for (int i = kk + 1; i < 16; ++i)
                x[i] = __builtin_fma(-L[i * LDT + kk], x[kk], x[i]);
            pin16(x);
        }
#pragma unroll
        for (int i = 0; i < 16; ++i)
            if (i > c)
                P[(16 * bp + i) * LDT + 16 * bp + c] = x[i];
    } else if (w == 1) {
        const T *U = S + 16 * bp * (LDT + 1);
        T x[16];
#pragma unroll
        for (int i = 0; i < 16; ++i)
            x[i] = (i == c) ? T(1) : T(0);
#pragma unroll
        for (int kk = 15; kk >= 0; --kk) {
            x[kk] *= rinv[16 * bp + kk];
#pragma unroll
            for (int i = 0; i < kk; ++i)
                x[i] = __builtin_fma(-U[i * LDT + kk], x[kk], x[i]);
            pin16(x);
        }
#pragma unroll
        for (int i = 0; i < 16; ++i)
            if (i <= c)
                P[(16 * bp + i) * LDT + 16 * bp + c] = x[i];
    }
    __syncthreads();
}

/* Diagonal block q of the inverse pack by one wave (lanes 0..15, one column
 * each): L_qq^{-1} (strict lower part, UPPER = false) or U_qq^{-1} (upper
 * part, UPPER = true) of a tile factored by tile_lu16, as tile_diag_inv16
 * forms them; put(i, c, v) receives element (i, c) of the block. */
template <typename T, bool UPPER, typename Put>
__device__ __forceinline__ void diag_block_inv(const T *S, const T *rinv, int q, Put &&put)
{
    const int c = launder(static_cast<int>(threadIdx.x) & 63);
    if (c >= 16)
        return;
    const T *D = S + 16 * q * (LDT + 1);
    T x[16];
#pragma unroll
    for (int i = 0; i < 16; ++i)
        x[i] = (i == c) ? T(1) : T(0);
    if (!UPPER) {
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
#pragma unroll
            for (int i = kk + 1; i < 16; ++i)
                x[i] = __builtin_fma(-D[i * LDT + kk], x[kk], x[i]);
            pin16(x);
        }
#pragma unroll
        for (int i = 0; i < 16; ++i)
            if (i > c)
                put(i, c, x[i]);
    } else {
#pragma unroll
        for (int kk = 15; kk >= 0; --kk) {
            x[kk] *= rinv[16 * q + kk];
#pragma unroll
            for (int i = 0; i < kk; ++i)
                x[i] = __builtin_fma(-D[i * LDT + kk], x[kk], x[i]);
            pin16(x);
        }
#pragma unroll
        for (int i = 0; i < 16; ++i)
            if (i <= c)
                put(i, c, x[i]);
    }
}

/*
 * Inverses of the factors of a tile factored by tile_lu16 (S, with 1/U_kk in
 * rinv): P (LDS, pitch LDT) receives L^{-1} in its strict lower part (its unit
 * diagonal implied) and U^{-1} in its upper part.  After the diagonal blocks
 * (tile_diag_inv16) the off-diagonal blocks follow one block diagonal at a
 * time on the matrix cores, from L X = I and U Y = I:
 *   X_ij = -X_ii sum_{k=j}^{i-1} L_ik X_kj   (i > j)
 *   Y_ij = -Y_ii sum_{k=i+1}^{j} U_ik Y_kj   (i < j).
 */
template <typename T>
__device__ __forceinline__ void tile_inv16(const T *S, const T *rinv, T *P)
{
    typedef typename vec4<T>::type V;
    tile_diag_inv16(S, rinv, P);
    S = launder(S);
    P = launder(P);
    const int t = threadIdx.x, w = wave_id();
    (void)t;
    /* diagonal blocks of the inverses, with the other factor's part masked
     * (loads unconditional, selects after: no divergent branches) */
    auto xdiag = [&](int bi, int r, int k) -> T {
        const T v = P[(16 * bi + r) * LDT + 16 * bi + k];
        return r > k ? v : (r == k ? T(1) : T(0));
    };
    auto ydiag = [&](int bi, int r, int k) -> T {
        const T v = P[(16 * bi + r) * LDT + 16 * bi + k];
        return r <= k ? v : T(0);
    };
#pragma unroll 1
    for (int d = 1; d < 4; ++d) {
        const int ntask = 2 * (4 - d);
        for (int task = w; task < ntask; task += 4) {
            const bool lower = task < 4 - d;
            const int a = lower ? task : task - (4 - d);
            V tacc = {0, 0, 0, 0};
            V x = {0, 0, 0, 0};
            if (lower) {
                const int i = a + d, j = a; /* T = sum_{k=j}^{i-1} L_ik X_kj */
                wave_mma16<T, 16>(
                    tacc, [&](int r, int k) { return S[(16 * i + r) * LDT + 16 * j + k]; },
                    [&](int k, int cc) { return xdiag(j, k, cc); });
                for (int kb = j + 1; kb < i; ++kb)
                    wave_mma16<T, 16>(
                        tacc, [&](int r, int k) { return S[(16 * i + r) * LDT + 16 * kb + k]; },
                        [&](int k, int cc) { return P[(16 * kb + k) * LDT + 16 * j + cc]; });
                wave_mma16_acc<T>(x, [&](int r, int k) { return -xdiag(i, r, k); }, tacc);
                acc_store<T>(x, P + 16 * i * LDT + 16 * j, LDT);
            } else {
                const int i = a, j = a + d; /* T = sum_{k=i+1}^{j} U_ik Y_kj */
                for (int kb = i + 1; kb < j; ++kb)
                    wave_mma16<T, 16>(
                        tacc, [&](int r, int k) { return S[(16 * i + r) * LDT + 16 * kb + k]; },
                        [&](int k, int cc) { return P[(16 * kb + k) * LDT + 16 * j + cc]; });
                wave_mma16<T, 16>(
                    tacc, [&](int r, int k) { return S[(16 * i + r) * LDT + 16 * j + k]; },
                    [&](int k, int cc) { return ydiag(j, k, cc); });
                wave_mma16_acc<T>(x, [&](int r, int k) { return -ydiag(i, r, k); }, tacc);
                acc_store<T>(x, P + 16 * i * LDT + 16 * j, LDT);
            }
        }
        __syncthreads();
    }
}

/*
 * 64 x 64 products on the matrix cores, in pieces: the workgroup's
 * accumulators (wave w holds the 32 x 32 quadrant (w / 2, w % 2) as 2 x 2
 * blocks of 16 x 16) are loaded from C, take acc (+|-)= A * B with
 * fa(r, k) = A[r][k] and fb(k, c) = B[k][c] read from LDS (inner size K),
 * and are stored.  `cref(r, c)` gives the address of C's element (r, c) or
 * nullptr outside the tile's valid part (read as zero, not written).
 */
template <typename T> struct Acc64 {
    typename vec4<T>::type v[2][2];
};
template <typename T, typename CRef> __device__ __forceinline__ void acc64_load(Acc64<T> &acc, const CRef &cref)
{
    const int w = wave_id(), l = threadIdx.x & 63, lr = l & 15, lk = l >> 4;
    const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const T *p = cref(wm + 16 * bi + acc_row<T>(lk, r), wn + 16 * bj + lr);
                acc.v[bi][bj][r] = p ? *p : T(0);
            }
}
template <typename T> __device__ __forceinline__ void acc64_zero(Acc64<T> &acc)
{
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                acc.v[bi][bj][r] = T(0);
}
template <typename T, typename CRef> __device__ __forceinline__ void acc64_store(const Acc64<T> &acc, const CRef &cref)
{
    const int w = wave_id(), l = threadIdx.x & 63, lr = l & 15, lk = l >> 4;
    const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                T *p = cref(wm + 16 * bi + acc_row<T>(lk, r), wn + 16 * bj + lr);
                if (p)
                    *p = acc.v[bi][bj][r];
            }
}
template <typename T, bool NEG, int K = TB, typename FA, typename FB>
__device__ __forceinline__ void acc64_mma(Acc64<T> &acc, FA &&fa, FB &&fb)
{
    const int w = wave_id(), l = threadIdx.x & 63, lr = l & 15, lk = l >> 4;
    const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
#pragma unroll 8
    for (int k = 0; k < K; k += 4) {
        T a[2], b[2];
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
            a[bi] = NEG ? -fa(wm + 16 * bi + lr, k + lk) : fa(wm + 16 * bi + lr, k + lk);
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
            b[bj] = fb(k + lk, wn + 16 * bj + lr);
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj)
                acc.v[bi][bj] = mfma16(a[bi], b[bj], acc.v[bi][bj]);
    }
}

/* acc64_mma restricted to the inner indices klo <= k < khi (multiples of 32,
 * uniform within the wave): the terms a triangular operand makes zero.  Each
 * 32-wide chunk is unrolled, so its operand reads are issued together. */
template <typename T, bool NEG, typename FA, typename FB>
__device__ __forceinline__ void acc64_mma_range(Acc64<T> &acc, FA &&fa, FB &&fb, int klo, int khi)
{
    const int w = wave_id(), l = threadIdx.x & 63, lr = l & 15, lk = l >> 4;
    const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
#pragma unroll 1
    for (int kc = klo; kc < khi; kc += 32)
#pragma unroll
        for (int k = kc; k < kc + 32; k += 4) {
            T a[2], b[2];
#pragma unroll
            for (int bi = 0; bi < 2; ++bi)
                a[bi] = NEG ? -fa(wm + 16 * bi + lr, k + lk) : fa(wm + 16 * bi + lr, k + lk);
#pragma unroll
            for (int bj = 0; bj < 2; ++bj)
                b[bj] = fb(k + lk, wn + 16 * bj + lr);
#pragma unroll
            for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                for (int bj = 0; bj < 2; ++bj)
                    acc.v[bi][bj] = mfma16(a[bi], b[bj], acc.v[bi][bj]);
        }
}

/* C = A * B (SET) or C -= A * B for one 64 x 64 tile (see above). */
template <typename T, bool SET, int K = TB, typename CRef, typename FA, typename FB>
__device__ __forceinline__ void wg_gemm64f(const CRef &cref, FA &&fa, FB &&fb)
{
    Acc64<T> acc;
    if (SET)
        acc64_zero(acc);
    else
        acc64_load(acc, cref);
    acc64_mma<T, !SET, K>(acc, fa, fb);
    acc64_store(acc, cref);
}

/* C addressing of a full 64 x 64 LDS tile (pitch LDT). */
template <typename T> struct LdsTile {
    T *S;
    __device__ __forceinline__ T *operator()(int r, int c) const { return S + r * LDT + c; }
};

/* Operand readers for the inverse pack P (LDS, pitch LDT) of tile_inv16. */
template <typename T> struct InvL { /* L^{-1}: strict lower of P, unit diagonal */
    const T *P;
    __device__ __forceinline__ T operator()(int r, int k) const
    {
        const T v = P[r * LDT + k];
        return r > k ? v : (r == k ? T(1) : T(0));
    }
};
template <typename T> struct InvU { /* U^{-1}: upper part of P */
    const T *P;
    __device__ __forceinline__ T operator()(int k, int c) const
    {
        const T v = P[k * LDT + c];
        return k <= c ? v : T(0);
    }
};

/* U^{-1} as a left operand: element (r, k) of the upper part of P. */
template <typename T> struct InvUFull {
    const T *P;
    __device__ __forceinline__ T operator()(int r, int k) const
    {
        const T v = P[r * LDT + k];
        return r <= k ? v : T(0);
    }
};

/* Load the nr x nc corner of the 64x64 tile at G into LDS S (pitch LDT), the
 * rest the identity (the padding a partial diagonal tile is factored with). */
template <typename T>
__device__ __forceinline__ void stage_tile_identity(T *S, const T *__restrict__ G, int64_t ldg, int nr, int nc)
{
    tile_xfer<T>([&](int r, int c) { return (r < nr && c < nc) ? G[(int64_t)r * ldg + c] : (r == c ? T(1) : T(0)); },
                 [&](int r, int c, T v) { S[r * LDT + c] = v; });
}

/*
 * acc -= A(nr x kw) * B(kw x nc) for one 64 x 64 tile held in the Acc64
 * accumulators (wave w: the 32 x 32 quadrant (w / 2, w % 2)), kw a multiple
 * of 16: the trailing updates of Eq. 6-c that a tile has pending, applied at
 * once.  Each wave loads its operands straight from memory into registers in
 * the matrix-core operand layout, 16 inner indices (a chunk) at a time, and
 * keeps two chunks in flight while it multiplies the third: no LDS, no
 * barrier, so the waves of a workgroup stream independently.  Within a chunk
 * lane group g = lane / 16 supplies inner indices 4g .. 4g+3 (one per
 * product), so a lane's four A elements are contiguous in memory.  Rows of A
 * past nr and columns of B past nc read as zero (their addresses clamped to
 * a valid element, the value then masked).  Ap = &A(0, 0) (pitch lda), Bp =
 * &B(0, 0) (pitch ldb).
 *
 * Every prefetch is issued, its chunk index clamped to the last chunk (the
 * last two re-read it from cache): with a prefetch behind a branch the
 * compiler's wait counts at the merge must cover the path that skipped it,
 * so the product before it waited for the chunk just requested as well.
 */
template <typename T, int NA = 1, int NB = 1> struct StreamRegs {
    T a[NA][2][4], b[NB][2][4];
    int k0; /* first inner index of the chunk (KMASK) */
};

/*
 * The same stream for NA x NB tiles that share their operands:
 * acc[ia * NB + ib] -= A_ia * B_ib, where A_ia is the 64-row block starting
 * 64 ia rows below Ap (nr[ia] valid rows) and B_ib the 64-column block
 * starting 64 ib columns right of Bp (nc[ib] valid columns).  Two tiles of
 * one block row (NB = 2) read their common left operand once, two tiles of
 * one block column (NA = 2) their common right operand: a quarter less
 * operand traffic than two separate streams.
 */
template <typename T, int NA, int NB, bool KMASK = false>
__device__ __forceinline__ void acc64_stream_n(Acc64<T> *acc, const T *Ap, int64_t lda, const T *Bp, int64_t ldb,
                                               const int (&nr)[NA], const int (&nc)[NB], int kw)
{
    /* KMASK: kw need not be a multiple of 16; inner indices past kw read as
     * zero (addresses clamped to kw - 1) */
    const int nch = KMASK ? (kw + 15) >> 4 : kw >> 4;
    if (nch == 0)
        return;
    const int w = wave_id(), l = threadIdx.x & 63, lr = l & 15, g = l >> 4;
    const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
    /* chunk 0's operands of this lane: A(r, 4g), B(4g, c) */
    const T *ap[NA][2];
    const T *bp[NB][2];
    bool aok[NA][2], bok[NB][2];
#pragma unroll
    for (int ia = 0; ia < NA; ++ia)
#pragma unroll
        for (int bi = 0; bi < 2; ++bi) {
            const int r = wm + 16 * bi + lr;
            aok[ia][bi] = r < nr[ia];
            ap[ia][bi] = Ap + (int64_t)(TB * ia + min(r, nr[ia] - 1)) * lda + 4 * g;
        }
#pragma unroll
    for (int ib = 0; ib < NB; ++ib)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) {
            const int c = wn + 16 * bj + lr;
            bok[ib][bj] = c < nc[ib];
            bp[ib][bj] = Bp + (int64_t)(4 * g) * ldb + TB * ib + min(c, nc[ib] - 1);
        }
    auto load = [&](StreamRegs<T, NA, NB> &R, int ci) {
        ci = min(ci, nch - 1);
        const int k0 = 16 * ci;
        R.k0 = k0;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            /* offset of inner index k0 + 4g + s from the lane's chunk-0 index */
            const int kk = KMASK ? min(k0 + 4 * g + s, kw - 1) - 4 * g : k0 + s;
#pragma unroll
            for (int ia = 0; ia < NA; ++ia)
#pragma unroll
                for (int bi = 0; bi < 2; ++bi)
                    R.a[ia][bi][s] = ap[ia][bi][kk];
#pragma unroll
            for (int ib = 0; ib < NB; ++ib)
#pragma unroll
                for (int bj = 0; bj < 2; ++bj)
                    R.b[ib][bj][s] = bp[ib][bj][(int64_t)kk * ldb];
        }
        /* keeps the loads here, ahead of the product after them: left free,
         * the compiler sinks them to their first use or moves the product
         * above them, and the chunk is waited for as soon as it is issued
         * (the operand pointers are not restrict-qualified, so that this
         * barrier may write what they point to) */
        asm volatile("" ::: "memory");
        __builtin_amdgcn_sched_barrier(0);
    };
    auto mul = [&](const StreamRegs<T, NA, NB> &R) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const bool kok = !KMASK || R.k0 + 4 * g + s < kw;
            T av[NA][2], bv[NB][2];
#pragma unroll
            for (int ia = 0; ia < NA; ++ia)
#pragma unroll
                for (int bi = 0; bi < 2; ++bi)
                    av[ia][bi] = (aok[ia][bi] && kok) ? -R.a[ia][bi][s] : T(0);
#pragma unroll
            for (int ib = 0; ib < NB; ++ib)
#pragma unroll
                for (int bj = 0; bj < 2; ++bj)
                    bv[ib][bj] = (bok[ib][bj] && kok) ? R.b[ib][bj][s] : T(0);
#pragma unroll
            for (int ia = 0; ia < NA; ++ia)
#pragma unroll
                for (int ib = 0; ib < NB; ++ib)
#pragma unroll
                    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                        for (int bj = 0; bj < 2; ++bj)
                            acc[ia * NB + ib].v[bi][bj] =
                                mfma16(av[ia][bi], bv[ib][bj], acc[ia * NB + ib].v[bi][bj]);
        }
    };
    if (NA * NB > 1) {
        /* a chunk of several tiles is multiplied long enough to cover the
         * next one's loads: one chunk in flight (and the registers of a
         * third set would spill) */
        StreamRegs<T, NA, NB> r0, r1;
        load(r0, 0);
        int c = 0;
        for (; c + 2 <= nch; c += 2) {
            load(r1, c + 1);
            mul(r0);
            load(r0, c + 2);
            mul(r1);
        }
        if (c < nch)
            mul(r0);
        return;
    }
    StreamRegs<T, NA, NB> r0, r1, r2;
    load(r0, 0);
    load(r1, 1);
    /* whole triples in a straight-line body (an exit between its products
     * would merge load states again), the last one or two chunks after */
    int c = 0;
    for (; c + 3 <= nch; c += 3) {
        load(r2, c + 2);
        mul(r0);
        load(r0, c + 3);
        mul(r1);
        load(r1, c + 4);
        mul(r2);
    }
    if (c < nch)
        mul(r0);
    if (c + 1 < nch)
        mul(r1);
}

template <typename T, bool KMASK = false>
__device__ __forceinline__ void acc64_stream(Acc64<T> &acc, const T *Ap, int64_t lda, const T *Bp, int64_t ldb, int nr,
                                             int nc, int kw)
{
    const int nrs[1] = {nr}, ncs[1] = {nc};
    acc64_stream_n<T, 1, 1, KMASK>(&acc, Ap, lda, Bp, ldb, nrs, ncs, kw);
}

/*
 * acc -= sum_t A_t B_t over a list of npairs pairs of 64 x 64 tiles (pitch
 * 64, the inner index fully inside the matrix): acc64_stream's chunk ring run
 * as one sequence over all the pairs, so that the first loads of each pair
 * are issued while the previous pair is multiplied instead of after it.
 * pair(t, A, B) sets the addresses of the t-th pair (uniform in the
 * workgroup); rows of A past nr and columns of B past nc read as zero.
 */
template <typename T, typename PairFn>
__device__ __forceinline__ void acc64_stream_pairs(Acc64<T> &acc, int npairs, PairFn &&pair, int nr, int nc)
{
    const int nch = 4 * npairs;
    if (nch == 0)
        return;
    const int w = wave_id(), l = threadIdx.x & 63, lr = l & 15, g = l >> 4;
    const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
    int aoff[2], boff[2];
    bool aok[2], bok[2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi) {
        const int r = wm + 16 * bi + lr;
        aok[bi] = r < nr;
        aoff[bi] = min(r, nr - 1) * TB + 4 * g;
    }
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
        const int c = wn + 16 * bj + lr;
        bok[bj] = c < nc;
        boff[bj] = 4 * g * TB + min(c, nc - 1);
    }
    auto load = [&](StreamRegs<T> &R, int ci) {
        ci = min(ci, nch - 1); /* every prefetch issued: see acc64_stream */
        const T *A;
        const T *B;
        pair(ci >> 2, A, B);
        const int k0 = 16 * (ci & 3);
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int s = 0; s < 4; ++s)
                R.a[0][bi][s] = A[aoff[bi] + k0 + s];
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int s = 0; s < 4; ++s)
                R.b[0][bj][s] = B[boff[bj] + (k0 + s) * TB];
        asm volatile("" ::: "memory");
        __builtin_amdgcn_sched_barrier(0);
    };
    auto mul = [&](const StreamRegs<T> &R) {
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                for (int bj = 0; bj < 2; ++bj)
                    acc.v[bi][bj] = mfma16(aok[bi] ? -R.a[0][bi][s] : T(0), bok[bj] ? R.b[0][bj][s] : T(0),
                                           acc.v[bi][bj]);
    };
    StreamRegs<T> r0, r1, r2;
    load(r0, 0);
    load(r1, 1); /* nch >= 4 */
    int c = 0; /* as in acc64_stream */
    for (; c + 3 <= nch; c += 3) {
        load(r2, c + 2);
        mul(r0);
        load(r0, c + 3);
        mul(r1);
        load(r1, c + 4);
        mul(r2);
    }
    if (c < nch)
        mul(r0);
    if (c + 1 < nch)
        mul(r1);
}

/*
 * Blocked Doolittle LU of one n x n system by one workgroup in Crout order
 * (Eq. 6-c's updates applied lazily): at block step j the diagonal tile and
 * the tiles of block row j and block column j receive, in one streamed
 * product each, every update of the steps before (K = 64 j), then
 *   - the diagonal tile is factored in LDS (tile_lu16, Eq. 6-a) and its
 *     factors inverted (tile_inv16),
 *   - block row j becomes U:   U_jc = L_jj^{-1} A_jc,
 *   - block column j becomes L: L_rj = A_rj U_jj^{-1},
 * all products on the matrix cores.  Every tile is read and written once
 * for its whole update.  With right-hand sides (B != NULL, n x nrhs, pitch
 * ldb) the forward substitution L Y = B (Eq. 1) rides along as extra columns
 * of block row j: Y_j = L_jj^{-1} (B_j - L_j,0:j Y_0:j).  Returns the first
 * zero pivot (1-based) or 0; the factor overwrites A, Y overwrites B.
 */
template <typename T>
__device__ __forceinline__ int wg_crout(T *__restrict__ A, int64_t lda, int n, T *__restrict__ B, int64_t ldb, int nrhs,
                                     TileSmem<T> &sm)
{
    const int nt = (n + TB - 1) / TB;
    int zero_at = 0;
    for (int j = 0; j < nt; ++j) {
        const int k0 = j * TB, kw = min(TB, n - k0);
        const T *Lrow = A + (int64_t)k0 * lda; /* L_j,0:j (rows k0.., columns 0..k0) */
        const T *Ucol = A + k0;                /* U_0:j,j (rows 0..k0, columns k0..) */
        /* diagonal tile: all pending updates, then into LDS with the
         * identity past the system's end */
        {
            Acc64<T> acc;
            T *Akk = A + (int64_t)k0 * lda + k0;
            acc64_load(acc, DenseC<T>{Akk, lda, kw, kw});
            acc64_stream(acc, Lrow, lda, Ucol, lda, kw, kw, k0);
            acc64_store(acc, LdsTile<T>{sm.t0});
            __syncthreads();
            if (threadIdx.x >= kw && threadIdx.x < TB)
                sm.t0[threadIdx.x * LDT + threadIdx.x] = T(1);
            __syncthreads();
            const int z = tile_lu16(sm.t0, sm.rinv, sm.aux, kw, &sm.zflag);
            if (z && !zero_at)
                zero_at = k0 + z;
            lds_store_tile(sm.t0, Akk, lda, kw, kw);
            if (j + 1 == nt && !B)
                break;
            tile_inv16(sm.t0, sm.rinv, sm.t1);
        }
        /* block row j right of the diagonal (U), then the right-hand sides
         * (Y); factor tiles two at a time where two remain (one stream for
         * both, the left operand read once) */
        const int ncol = nt - 1 - j + (B ? (nrhs + TB - 1) / TB : 0);
        for (int q = 0; q < ncol; ++q) {
            if (q + 1 < nt - 1 - j) {
                const int c0 = k0 + TB + q * TB, cw1 = min(TB, n - c0 - TB);
                T *G = A + (int64_t)k0 * lda + c0;
                const int nrs[1] = {kw}, ncs[2] = {TB, cw1};
                Acc64<T> acc[2];
                acc64_load(acc[0], DenseC<T>{G, lda, kw, TB});
                acc64_load(acc[1], DenseC<T>{G + TB, lda, kw, cw1});
                acc64_stream_n<T, 1, 2>(acc, Lrow, lda, A + c0, lda, nrs, ncs, k0);
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    acc64_store(acc[h], LdsTile<T>{sm.t0});
                    __syncthreads();
                    wg_gemm64f<T, true>(DenseC<T>{G + h * TB, lda, kw, h ? cw1 : TB}, InvL<T>{sm.t1},
                                        [&](int k, int c) { return sm.t0[k * LDT + c]; });
                    __syncthreads();
                }
                ++q;
                continue;
            }
            const bool rhs = q >= nt - 1 - j;
            const int c0 = rhs ? (q - (nt - 1 - j)) * TB : k0 + TB + q * TB;
            const int cw = min(TB, (rhs ? nrhs : n) - c0);
            T *G = rhs ? B + (int64_t)k0 * ldb + c0 : A + (int64_t)k0 * lda + c0;
            const int64_t ldg = rhs ? ldb : lda;
            const T *Bop = rhs ? B + c0 : A + c0;
            Acc64<T> acc;
            acc64_load(acc, DenseC<T>{G, ldg, kw, cw});
            acc64_stream(acc, Lrow, lda, Bop, ldg, kw, cw, k0);
            acc64_store(acc, LdsTile<T>{sm.t0});
            __syncthreads();
            wg_gemm64f<T, true>(DenseC<T>{G, ldg, kw, cw}, InvL<T>{sm.t1},
                                [&](int k, int c) { return sm.t0[k * LDT + c]; });
            __syncthreads();
        }
        /* block column j below the diagonal (L), two tiles at a time where
         * two remain (the right operand read once) */
        for (int r = j + 1; r < nt; ++r) {
            if (r + 1 < nt) {
                const int r0 = r * TB, rw1 = min(TB, n - r0 - TB);
                T *G = A + (int64_t)r0 * lda + k0;
                const int nrs[2] = {TB, rw1}, ncs[1] = {kw};
                Acc64<T> acc[2];
                acc64_load(acc[0], DenseC<T>{G, lda, TB, kw});
                acc64_load(acc[1], DenseC<T>{G + (int64_t)TB * lda, lda, rw1, kw});
                acc64_stream_n<T, 2, 1>(acc, A + (int64_t)r0 * lda, lda, Ucol, lda, nrs, ncs, k0);
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    acc64_store(acc[h], LdsTile<T>{sm.t0});
                    __syncthreads();
                    wg_gemm64f<T, true>(DenseC<T>{G + (int64_t)h * TB * lda, lda, h ? rw1 : TB, kw},
                                        [&](int rr, int k) { return sm.t0[rr * LDT + k]; }, InvU<T>{sm.t1});
                    __syncthreads();
                }
                ++r;
                continue;
            }
            const int r0 = r * TB, rw = min(TB, n - r0);
            T *G = A + (int64_t)r0 * lda + k0;
            Acc64<T> acc;
            acc64_load(acc, DenseC<T>{G, lda, rw, kw});
            acc64_stream(acc, A + (int64_t)r0 * lda, lda, Ucol, lda, rw, kw, k0);
            acc64_store(acc, LdsTile<T>{sm.t0});
            __syncthreads();
            wg_gemm64f<T, true>(DenseC<T>{G, lda, rw, kw}, [&](int rr, int k) { return sm.t0[rr * LDT + k]; },
                                InvU<T>{sm.t1});
            __syncthreads();
        }
    }
    __syncthreads();
    return zero_at;
}

/* ------------------------------------------------ workgroup-level LU --- */

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


/*
 * Exchange between the workgroups of a multi-workgroup solve.  Blocks are
 * solved in a fixed order and each workgroup, after storing its block,
 * raises a shared counter `solved` to (its position + 1); a workgroup that
 * needs the block at position d waits for solved > d.  The solved values
 * are stored and loaded with device-coherent (agent-scope) atomic
 * operations, which go to the point of coherence instead of the caches of
 * one XCD, so neither side needs cache write-back or invalidation: a
 * producer that signals through a counter first waits for its own stores to
 * complete (s_waitcnt).
 */
template <typename T> __device__ __forceinline__ T load_coherent(const T *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T> __device__ __forceinline__ void store_coherent(T *p, T v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

/* Bookkeeping of every bounded wait, called once per spin: true when the
 * waiter must stop waiting -- after `limit` spins (it then ORs 1 into the
 * status word) or as soon as any waiter of the call has given up (the status
 * word is re-read every 64 spins).  One lost producer therefore ends all the
 * waits of a call within a few hundred spins each instead of a full budget
 * per wait, and the launches drain. */
__device__ __forceinline__ bool wait_give_up(int *status, long spins, long limit)
{
    if (spins > limit) {
        atomicOr(status, 1);
        __threadfence();
        return true;
    }
    return (spins & 63) == 63 && load_coherent(status) != 0;
}

/* Wait until *solved > d (thread 0 polls, at most `limit` spins; the value
 * seen is kept in *avail so later positions below it need no poll); every
 * thread returns after the workgroup barrier. */
__device__ __forceinline__ void wait_solved(const int *solved, int d, int *avail, int *status, long limit)
{
    if (threadIdx.x == 0 && *avail <= d) {
        int a = *avail;
        long spins = 0;
        while ((a = __hip_atomic_load(solved, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) <= d) {
            __builtin_amdgcn_s_sleep(1);
            if (wait_give_up(status, ++spins, limit)) {
                a = d + 1;
                break;
            }
        }
        *avail = a;
    }
    __syncthreads();
}

/* Marker of a value not yet produced in an exchange buffer: a signaling
 * NaN, which no arithmetic result can be (operations return quiet NaNs), so
 * a value read as anything else is final. */
__device__ __forceinline__ bool is_unsolved_mark(double x) { return __double_as_longlong(x) == 0x7FF40000DEADBEEFll; }
__device__ __forceinline__ bool is_unsolved_mark(float x) { return __float_as_int(x) == 0x7FA0BEEF; }
constexpr unsigned long long kUnsolvedMark64 = 0x7FF40000DEADBEEFull;
constexpr unsigned int kUnsolvedMark32 = 0x7FA0BEEFu;

/*
 * Solve one 64-row block `blk` of op(T) Y = B (Eq. 1's forward or backward
 * substitution, blocked): accumulate the contributions of the blocks solved
 * before it (at most `maxdep` of them, the earliest solved first), then solve
 * with the diagonal block.  NR <= 8 columns of B are handled (nrhs_here of
 * them valid), all by the calling workgroup.  `op(S, bi, bj)` stages
 * operator blocks.
 *
 * Thread t handles row rr = t / 4; for the off-diagonal products its quarter
 * q = t % 4 covers 16 of the 64 columns and the four partial sums are joined
 * with wavefront shuffles.
 */
template <typename T, int MODE, int NR, typename Op>
__device__ void solve_block(const Op &op, int n, T *__restrict__ B, int64_t ldb, int nrhs_here, int blk,
                            int maxdep, TileSmem<T> &sm)
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
    /* this block's own right-hand side, loaded before any wait (no other
     * workgroup writes these rows) */
    T rhs[NR];
#pragma unroll
    for (int c = 0; c < NR; ++c)
        rhs[c] = (q == 0 && rr < nr && c < nrhs_here) ? B[(int64_t)(r0 + rr) * ldb + c] : T(0);
    if (ndep > 0)
        op.seg(blk, FWD ? blk - ndep : blk + ndep, rr, q, mc);
    for (int d = 0; d < ndep; ++d) {
        const int j = FWD ? blk - ndep + d : blk + ndep - d;
        const int jw = min(TB, n - j * TB);
        if (d + 1 < ndep)
            op.seg(blk, FWD ? j + 1 : j - 1, rr, q, mn);
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
            Y[rr * NR + c] = rhs[c] - acc[c];
    op(sm.t0, blk, blk);
    __syncthreads();
    /* diagonal block: wave w sweeps it for the right-hand sides w, w + NW, ...,
     * lane r holding row r; the finished row's values are broadcast with
     * readlane, so no barrier is needed */
    constexpr int NW = NR < 4 ? NR : 4, CPW = NR / NW;
    const int w = wave_id();
    if (w < NW) {
        const T *M = sm.t0;
        const int r = t & 63;
        T y[CPW];
#pragma unroll
        for (int j = 0; j < CPW; ++j)
            y[j] = Y[r * NR + w + NW * j];
        const T rin = (!tri_unit(MODE) && r < nr) ? recip(M[r * LDT + r]) : T(1);
        for (int s = 0; s < nr; ++s) {
            const int m = FWD ? s : nr - 1 - s;
            const bool after = FWD ? (r > m) : (r < m);
            const T cf = after ? M[r * LDT + m] : T(0);
#pragma unroll
            for (int j = 0; j < CPW; ++j) {
                if (!tri_unit(MODE))
                    y[j] = (r == m) ? y[j] * rin : y[j];
                const T ym = bcast(y[j], m);
                y[j] = __builtin_fma(-cf, ym, y[j]);
            }
        }
        if (r < nr)
#pragma unroll
            for (int j = 0; j < CPW; ++j)
                if (w + NW * j < nrhs_here)
                    B[(int64_t)(r0 + r) * ldb + w + NW * j] = y[j];
    }
    __syncthreads();
}

/*
 * A wave's pass over rows of a row-major matrix M (pitch ld), four rows at a
 * time: items are (group g of four rows starting at row0(g), 256-column block
 * of [c0, c1)); lane l loads rows row0(g) + u, columns cb + 64 m + l (u, m <
 * 4; indices clamped to nrows - 1 and c1 - 1, so every load is valid and the
 * consumer masks) one item ahead of the item it consumes, so that a load's
 * latency overlaps the previous item instead of stalling each one.
 * consume(g, cb, v) receives an item's values, finish(g) follows a group's
 * last column block.  Nothing happens when c1 <= c0 or ngroups <= 0.
 */
template <typename T, typename RowOf, typename Consume, typename Finish>
__device__ __forceinline__ void wave_rows4_stream(const T *__restrict__ M, int64_t ld, int ngroups, RowOf &&row0,
                                                  int nrows, int c0, int c1, Consume &&consume, Finish &&finish)
{
    const int l = threadIdx.x & 63;
    const int ncb = c1 > c0 ? (c1 - c0 + 255) >> 8 : 0;
    const int total = ngroups > 0 ? ngroups * ncb : 0;
    if (total == 0)
        return;
    auto load = [&](int it, T (&v)[4][4]) {
        const int g = it / ncb, cb = c0 + ((it - g * ncb) << 8), r = row0(g);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const T *rp = M + (int64_t)min(r + u, nrows - 1) * ld;
#pragma unroll
            for (int m = 0; m < 4; ++m)
                v[u][m] = rp[min(cb + 64 * m + l, c1 - 1)];
        }
    };
    auto step = [&](int it, const T (&v)[4][4]) {
        const int g = it / ncb, cbi = it - g * ncb;
        consume(g, c0 + (cbi << 8), v);
        if (cbi == ncb - 1)
            finish(g);
    };
    T va[4][4], vb[4][4];
    load(0, va);
#pragma unroll 1
    for (int it = 0; it < total; it += 2) {
        load(min(it + 1, total - 1), vb); /* unconditional: no branch around the loads */
        step(it, va);
        if (it + 1 >= total)
            break;
        load(min(it + 2, total - 1), va);
        step(it + 1, vb);
    }
}

/*
 * Triangular solve of op(T) x = b with ONE right-hand side by one workgroup,
 * x held in LDS (xs, in place, n elements): MODE TRI_L (L unit lower,
 * forward substitution), TRI_U (U upper, backward), or their transposes
 * TRI_UT (U^T, forward) and TRI_LT (L^T, backward), Eq. 1.  Block by block
 * (64 rows of op(T)), in solve order:
 *   1. the block row's product with the part of x already solved, read
 *      straight from the factor with coalesced loads, while the 64 x 64
 *      diagonal block is fetched into registers for LDS (tri, pitch LDT):
 *      L and U by rows (a GEMV: wave w takes rows 16w .. 16w+15 of the
 *      block, four at a time, its lanes the columns, all of a group's loads
 *      issued before its sums, reduced with wavefront shuffles); U^T and L^T
 *      by the columns of T (lane l the column, wave w every fourth solved
 *      row, 16 rows' loads in flight ahead of their sums, the four waves'
 *      sums added through LDS);
 *   2. the diagonal triangle by wave 0 (lane r holds row r; each finished
 *      value is broadcast with readlane, no barrier).
 * The vector never leaves LDS.  Ends with a barrier.
 */
template <typename T, int MODE>
__device__ __forceinline__ void wg_trsv1(const T *__restrict__ LU, int64_t lda, int n, T *xs, T *tri)
{
    constexpr bool FWD = tri_forward(MODE), UNIT = tri_unit(MODE), TRANS = tri_trans(MODE);
    const int nb = (n + TB - 1) / TB;
    const int t = threadIdx.x, w = wave_id(), l = t & 63;
    for (int step = 0; step < nb; ++step) {
        const int blk = FWD ? step : nb - 1 - step;
        const int r0 = blk * TB, rw = min(TB, n - r0);
        const int c0 = FWD ? 0 : r0 + rw, c1 = FWD ? r0 : n; /* solved columns of op(T) */
        /* diagonal block: loads issued now, parked in LDS after the product */
        T dv[16];
        {
            /* unconditional loads (clamped), masked when parked */
            const int c = min(l, rw - 1);
#pragma unroll
            for (int i = 0; i < 16; ++i)
                dv[i] = LU[(int64_t)(r0 + min(w + 4 * i, rw - 1)) * lda + r0 + c];
        }
        if (!TRANS) {
            /* GEMV of the block row with the solved part, 4 rows at a time,
             * loads one item ahead */
            T sum[4] = {T(0), T(0), T(0), T(0)};
            wave_rows4_stream<T>(
                LU + (int64_t)r0 * lda, lda, 4, [&](int g) { return 16 * w + 4 * g; }, rw, c0, c1,
                [&](int, int cb, const T(&v)[4][4]) {
                    T xv[4];
#pragma unroll
                    for (int m = 0; m < 4; ++m) {
                        const int c = cb + 64 * m + l;
                        xv[m] = c < c1 ? xs[c] : T(0);
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u)
#pragma unroll
                        for (int m = 0; m < 4; ++m)
                            sum[u] = __builtin_fma(v[u][m], xv[m], sum[u]);
                },
                [&](int g) {
                    const int rbase = 16 * w + 4 * g;
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
#pragma unroll
                        for (int o = 32; o > 0; o >>= 1)
                            sum[u] += __shfl_xor(sum[u], o);
                        if (l == 0 && rbase + u < rw)
                            xs[r0 + rbase + u] -= sum[u];
                        sum[u] = T(0);
                    }
                });
        } else if (c1 > c0) {
            /* sum over the solved rows k of T of T[k][r0 + l] x[k]: wave w
             * the rows c0 + w + 4j, RB of them per item, one item's loads in
             * flight while the previous one is summed (addresses clamped,
             * rows past c1 masked at use) */
            constexpr int RB = 16;
            const int nit = (c1 - c0 + 4 * RB - 1) / (4 * RB);
            const T *col = LU + r0 + min(l, rw - 1);
            T acc = T(0);
            auto load = [&](int it, T(&v)[RB]) {
#pragma unroll
                for (int u = 0; u < RB; ++u)
                    v[u] = col[(int64_t)min(c0 + 4 * (it * RB + u) + w, n - 1) * lda];
            };
            auto use = [&](int it, const T(&v)[RB]) {
#pragma unroll
                for (int u = 0; u < RB; ++u) {
                    const int k = c0 + 4 * (it * RB + u) + w;
                    const T a = __builtin_fma(v[u], xs[min(k, n - 1)], acc);
                    acc = k < c1 ? a : acc;
                }
            };
            T va[RB], vb[RB];
            load(0, va);
#pragma unroll 1
            for (int it = 0; it < nit; it += 2) {
                load(min(it + 1, nit - 1), vb); /* unconditional: no branch around the loads */
                use(it, va);
                if (it + 1 >= nit)
                    break;
                load(min(it + 2, nit - 1), va);
                use(it + 1, vb);
            }
            tri[w * LDT + l] = acc;
            __syncthreads();
            if (w == 0 && l < rw)
                xs[r0 + l] -= (tri[l] + tri[LDT + l]) + (tri[2 * LDT + l] + tri[3 * LDT + l]);
            __syncthreads(); /* tri is rewritten below */
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int r = w + 4 * i;
            const T v = (r < rw && l < rw) ? dv[i] : T(0);
            if (TRANS)
                tri[l * LDT + r] = v; /* op(T) = T^T: element (l, r) */
            else
                tri[r * LDT + l] = v;
        }
        __syncthreads();
        /* the triangle: wave 0, lane r holds row r */
        if (w == 0) {
            const int r = l;
            T y = r < rw ? xs[r0 + r] : T(0);
            const T rin = (!UNIT && r < rw) ? recip(tri[r * LDT + r]) : T(1);
            if (rw == TB) {
                /* a full block: unrolled in chunks of 16 steps, each chunk's
                 * coefficients read before its chain starts */
#pragma unroll
                for (int s0 = 0; s0 < TB; s0 += 16) {
                    T cf[16];
#pragma unroll
                    for (int i = 0; i < 16; ++i) {
                        const int m = FWD ? s0 + i : TB - 1 - s0 - i;
                        const T c = tri[r * LDT + m];
                        cf[i] = (FWD ? (r > m) : (r < m)) ? c : T(0);
                    }
#pragma unroll
                    for (int i = 0; i < 16; ++i) {
                        const int m = FWD ? s0 + i : TB - 1 - s0 - i;
                        if (!UNIT)
                            y = (r == m) ? y * rin : y;
                        y = __builtin_fma(-cf[i], bcast(y, m), y);
                    }
                }
            } else {
                for (int s = 0; s < rw; ++s) {
                    const int m = FWD ? s : rw - 1 - s;
                    const bool after = FWD ? (r > m) : (r < m);
                    const T cf = after ? tri[r * LDT + m] : T(0);
                    if (!UNIT)
                        y = (r == m) ? y * rin : y;
                    const T ym = bcast(y, m);
                    y = __builtin_fma(-cf, ym, y);
                }
            }
            if (r < rw)
                xs[r0 + r] = y;
        }
        __syncthreads();
    }
}

/* Whole triangular solve of op(T) by one workgroup, block after block. */
template <typename T, int MODE, int NR>
__device__ void wg_solve(const T *LU, int64_t lda, int n, T *B, int64_t ldb, int nrhs_here, TileSmem<T> &sm)
{
    const int nb = (n + TB - 1) / TB;
    const DenseOp<T, MODE> op{LU, lda, n};
    for (int s = 0; s < nb; ++s) {
        const int blk = tri_forward(MODE) ? s : nb - 1 - s;
        solve_block<T, MODE, NR>(op, n, B, ldb, nrhs_here, blk, nb, sm);
    }
}

} /* namespace ebv */

#endif /* EBV_DEVICE_HPP */
