/*
 * EbV ownership map: which work unit owns which row (or column, tile, system).
 *
 * The paper splits L into its n column vectors and U into its n row vectors
 * (the "bi-vectorization") and then joins the first vector with the last, the
 * second with the second-to-last, and so on, so that every joined vector has
 * the same length and every thread gets the same amount of work ("Equal
 * bi-vectorized" section, Eq. 7 and the paragraph after it).  Vector i (1-based)
 * of L has length n - i, vector n - i has length i: joined, n.
 *
 * In a right-looking step k only rows k+1..n-1 are still active.  Giving unit u
 * the joined pair {v, n-1-v} (0-based) keeps every unit's share of every step's
 * rank-1 update within one row of the mean; with several pairs per unit the
 * pairs are dealt out round-robin.  This header is plain C++ so that the host
 * test-suite can check those properties without a GPU.
 */
#ifndef EBV_PAIRING_H
#define EBV_PAIRING_H

#if defined(__HIPCC__)
#define EBV_HD __host__ __device__ __forceinline__
#else
#define EBV_HD inline
#endif

/* Partner of vector i among n vectors (0-based): first with last. */
EBV_HD constexpr int ebv_partner(int i, int n) { return n - 1 - i; }

/* Row owned by unit u (0..units-1) in slot q (0..2*(n/(2*units))-1) when n
 * rows are shared by `units` units: slot pairs (2p, 2p+1) hold the joined
 * vectors v = u + units*p and n-1-v. */
EBV_HD constexpr int ebv_row(int u, int q, int units, int n)
{
    return (q & 1) ? (n - 1 - (u + units * (q >> 1))) : (u + units * (q >> 1));
}

/* Inverse of ebv_row for the layout used by the register tiles: n = 64 rows,
 * 16 units, 4 slots per unit.  Returns unit*4 + slot. */
EBV_HD constexpr int ebv_owner64(int i)
{
    return (i < 16) ? (i * 4 + 0)
         : (i < 32) ? ((i - 16) * 4 + 2)
         : (i < 48) ? ((47 - i) * 4 + 3)
                    : ((63 - i) * 4 + 1);
}

/* Position of system rank r in the EbV batch order: the largest system first,
 * then the smallest, then the second largest, the second smallest, ...
 * Given systems sorted by decreasing cost (index 0 = largest), slot r of the
 * schedule takes sorted index ebv_batch_slot(r, count). */
EBV_HD constexpr int ebv_batch_slot(int r, int count)
{
    return (r & 1) ? (count - 1 - (r >> 1)) : (r >> 1);
}

#endif /* EBV_PAIRING_H */
