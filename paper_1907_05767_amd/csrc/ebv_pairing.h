/*
 * EbV pairing map: which units of work are joined.
 *
 * The paper splits L into its n column vectors and U into its n row vectors
 * (the "bi-vectorization") and then joins the first vector with the last, the
 * second with the second-to-last, and so on, so that every joined vector has
 * the same length and every thread gets the same amount of work ("Equal
 * bi-vectorized" section, Eq. 7 and the paragraph after it).  Vector i (1-based)
 * of L has length n - i, vector n - i has length i: joined, n.
 *
 * The same rule applies to any set of work units of unequal cost: pairing the
 * costliest with the cheapest equalizes the totals.  The ragged batch uses it
 * at system granularity (ebv_batch_slot, through ebv_batched_order).  Inside
 * one dense factorization the blocked schedule gives every tile the same
 * work already, so no pairing is applied there.  This header is plain C++ so
 * that the host test-suite can check its properties without a GPU.
 */
#ifndef EBV_PAIRING_H
#define EBV_PAIRING_H

#if defined(__HIPCC__)
#define EBV_HD __host__ __device__ __forceinline__
#else
#define EBV_HD inline
#endif

/* Position of system rank r in the EbV batch order: the largest system first,
 * then the smallest, then the second largest, the second smallest, ...
 * Given systems sorted by decreasing cost (index 0 = largest), slot r of the
 * schedule takes sorted index ebv_batch_slot(r, count). */
EBV_HD constexpr int ebv_batch_slot(int r, int count)
{
    return (r & 1) ? (count - 1 - (r >> 1)) : (r >> 1);
}

#endif /* EBV_PAIRING_H */
