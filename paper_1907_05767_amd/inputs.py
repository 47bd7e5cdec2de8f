"""Seeded synthetic inputs shared by the GPU path's tests/bench and the CPU oracle.

This module draws random numbers and lays them out; it performs none of the
solver's arithmetic (no elimination, no substitution).  Both sides receive the
arrays it returns, so neither needs to import the other.

Problem class: the paper's Eq. (2) shows a unit-diagonal, diagonally dominant
coefficient matrix, for which LU needs no pivoting.  The recipe used here:

* off-diagonal entries a_ij ~ U(-1, 1), drawn row by row;
* each row i is scaled so that sum_{j != i} |a_ij| == s (s < 1), and a_ii = 1,
  so every row is strictly diagonally dominant with margin 1 - s;
* right-hand sides and loss weights are iid N(0, 1).

Everything is drawn from numpy's PCG64 generator with an explicit seed.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "dense",
    "rhs",
    "band",
    "band_to_dense",
    "ragged",
    "ragged_sizes",
    "uniform_batch",
    "skyline",
    "skyline_to_dense",
]


def _scale_rows(off: np.ndarray, s: float) -> np.ndarray:
    """Scale each row of ``off`` (diagonal already zero) to absolute sum ``s``."""
    rs = np.abs(off).sum(axis=1)
    rs[rs == 0.0] = 1.0
    return off * (s / rs)[:, None]


def dense(n: int, s: float = 0.5, seed: int = 0, dtype=np.float64) -> np.ndarray:
    """Dense n x n unit-diagonal matrix with off-diagonal row |sum| = s (row-major)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if n == 0:
        return np.zeros((0, 0), dtype=dtype)
    off = rng.uniform(-1.0, 1.0, size=(n, n))
    np.fill_diagonal(off, 0.0)
    a = _scale_rows(off, s)
    np.fill_diagonal(a, 1.0)
    return np.ascontiguousarray(a, dtype=dtype)


def rhs(n: int, nrhs: int = 1, seed: int = 0, dtype=np.float64) -> np.ndarray:
    """n x nrhs right-hand side, iid N(0,1), row-major (b_ic at [i, c])."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.ascontiguousarray(rng.standard_normal((n, nrhs)), dtype=dtype)


def band(n: int, kl: int, ku: int, s: float = 0.5, seed: int = 0) -> np.ndarray:
    """Band matrix in row-wise band storage.

    Returns AB of shape (n, kl + ku + 1) with AB[i, j - i + kl] = a_ij for
    max(0, i - kl) <= j <= min(n - 1, i + ku); every other slot is zero.
    Only entries inside the band are drawn; each row's in-band off-diagonal
    absolute sum is scaled to ``s`` and the diagonal is 1.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    w = kl + ku + 1
    ab = rng.uniform(-1.0, 1.0, size=(n, w))
    i = np.arange(n)[:, None]
    j = i + np.arange(w)[None, :] - kl
    inside = (j >= 0) & (j < n)
    ab[~inside] = 0.0
    ab[:, kl] = 0.0
    ab = _scale_rows(ab, s)
    ab[:, kl] = 1.0
    return np.ascontiguousarray(ab)


def band_to_dense(ab: np.ndarray, kl: int, ku: int) -> np.ndarray:
    """Expand row-wise band storage (see ``band``) into a dense row-major matrix."""
    n, w = ab.shape
    assert w == kl + ku + 1
    a = np.zeros((n, n), dtype=ab.dtype)
    for i in range(n):
        lo, hi = max(0, i - kl), min(n - 1, i + ku)
        a[i, lo:hi + 1] = ab[i, lo - i + kl:hi - i + kl + 1]
    return a


def ragged_sizes(count: int, nmin: int, nmax: int, seed: int) -> np.ndarray:
    """System sizes n_s ~ U{nmin..nmax} (inclusive), int32."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(nmin, nmax + 1, size=count).astype(np.int32)


def ragged(count: int, nmin: int, nmax: int, s: float = 0.5, seed: int = 0, nrhs: int = 1):
    """Packed ragged batch of independent systems.

    Returns (n, offA, A, offB, B):
      n     int32[count]   system sizes ~ U{nmin..nmax}
      offA  int64[count]   element offset of system s in A (row-major n_s x n_s, lda = n_s)
      A     float64[sum n_s^2]
      offB  int64[count]   element offset of system s in B (row-major n_s x nrhs)
      B     float64[sum n_s * nrhs]
    System s is drawn with seed sequence child s of ``seed``.
    """
    ns = ragged_sizes(count, nmin, nmax, seed)
    children = np.random.SeedSequence(seed).spawn(count)
    offA = np.zeros(count, dtype=np.int64)
    offB = np.zeros(count, dtype=np.int64)
    if count:
        offA[1:] = np.cumsum(ns.astype(np.int64) ** 2)[:-1]
        offB[1:] = np.cumsum(ns.astype(np.int64) * nrhs)[:-1]
    totA = int((ns.astype(np.int64) ** 2).sum())
    totB = int(ns.astype(np.int64).sum() * nrhs)
    A = np.empty(totA, dtype=np.float64)
    B = np.empty(totB, dtype=np.float64)
    for k in range(count):
        sub = children[k].generate_state(2)
        n = int(ns[k])
        A[offA[k]:offA[k] + n * n] = dense(n, s, int(sub[0])).ravel()
        B[offB[k]:offB[k] + n * nrhs] = rhs(n, nrhs, int(sub[1])).ravel()
    return ns, offA, A, offB, B


def uniform_batch(batch: int, n: int, s: float = 0.5, seed: int = 0, nrhs: int = 1):
    """(batch, n, n) matrices and (batch, n, nrhs) right-hand sides; system k uses
    seed-sequence child k of ``seed``."""
    children = np.random.SeedSequence(seed).spawn(batch)
    A = np.empty((batch, n, n), dtype=np.float64)
    B = np.empty((batch, n, nrhs), dtype=np.float64)
    for k in range(batch):
        sub = children[k].generate_state(2)
        A[k] = dense(n, s, int(sub[0]))
        B[k] = rhs(n, nrhs, int(sub[1]))
    return A, B


def skyline(n: int, wshort: int = 64, wlong: int = 1024, plong: float = 0.1, s: float = 0.5, seed: int = 0):
    """Skyline (profile) matrix: a variable-bandwidth stand-in for the paper's
    "sparse" systems (Table 1, structure unstated).

    Row i's lower profile starts at column f_i = max(0, i - wl_i), column j's
    upper profile at row g_j = max(0, j - wu_j); each width is drawn
    independently, U{1..wshort} with probability 1 - plong and U{wshort..wlong}
    otherwise (a few tall columns and long rows, as in skyline matrices of
    structural problems).  Entries inside the profile are U(-1, 1); each row's
    off-diagonal absolute sum is scaled to s and the diagonal is 1.

    Storage (the classic skyline layout): the strictly lower part by rows, row
    i holding a_ij for f_i <= j < i at AL[rp[i] + j - f_i]; the upper part
    with the diagonal by columns, column j holding a_ij for g_j <= i <= j at
    AU[cp[j] + i - g_j] (the diagonal last).  Returns (f, rp, AL, g, cp, AU)
    with f, g int32[n] and rp, cp int64[n + 1].
    """
    rng = np.random.Generator(np.random.PCG64(seed))

    def widths():
        tall = rng.uniform(size=n) < plong
        w = np.where(tall, rng.integers(wshort, wlong + 1, size=n), rng.integers(1, wshort + 1, size=n))
        return w.astype(np.int64)

    idx = np.arange(n, dtype=np.int64)
    f = np.maximum(0, idx - widths()).astype(np.int32)
    g = np.maximum(0, idx - widths()).astype(np.int32)
    rp = np.zeros(n + 1, dtype=np.int64)
    cp = np.zeros(n + 1, dtype=np.int64)
    rp[1:] = np.cumsum(idx - f)
    cp[1:] = np.cumsum(idx - g + 1)
    AL = rng.uniform(-1.0, 1.0, size=int(rp[-1]))
    AU = rng.uniform(-1.0, 1.0, size=int(cp[-1]))
    # row of every upper entry, and the off-diagonal absolute sum of each row
    urow = np.concatenate([np.arange(g[j], j + 1) for j in range(n)]) if n else np.zeros(0, np.int64)
    diag = cp[1:] - 1
    AU[diag] = 0.0
    lrow = np.repeat(idx, idx - f)
    rs = np.zeros(n)
    np.add.at(rs, lrow, np.abs(AL))
    np.add.at(rs, urow, np.abs(AU))
    rs[rs == 0.0] = 1.0
    AL *= (s / rs)[lrow]
    AU *= (s / rs)[urow]
    AU[diag] = 1.0
    return f, rp, AL, g, cp, AU


def skyline_to_dense(f, rp, AL, g, cp, AU) -> np.ndarray:
    """Expand skyline storage (see ``skyline``) into a dense row-major matrix."""
    n = len(f)
    a = np.zeros((n, n))
    for i in range(n):
        a[i, f[i]:i] = AL[rp[i]:rp[i + 1]]
    for j in range(n):
        a[g[j]:j + 1, j] = AU[cp[j]:cp[j + 1]]
    return a
