"""Counter-based random numbers for the sketch matrices (test infrastructure).

Every node of the distributed method draws the same random sketch S^t from a
shared seed (Sec. 3.4, the paragraph after the B^t all-reduce, and Alg. 2).
The paper does not name a generator; this oracle and the HIP path each
implement Philox4x32-10 from its published definition (Salmon, Moraes, Dror,
Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11), so that S^t is a
pure function of (seed, t, side, row, column) and the two implementations can
be compared bit for bit on the integer stream.

Counter layout (a reading of the paper, which leaves it open):
    counter = (q, j, side | kind << 8, t), key = (seed mod 2^32, seed >> 32)
where j is the row of S (an index into the long dimension), q groups four
consecutive sketch columns, side 0 is the U-subproblem (S^t, n x d) and side 1
the V-subproblem (S'^t, m x d'), kind 0 is Gaussian, 1 subsampling, 2 the
count sketch's bucket and sign, 3 the SRHT's signs and 4 the SRHT's sampled
Hadamard columns.  The counters use the row index j of the whole matrix: a
block of rows of S (one node's share of the long dimension) is the same
block of the full sketch.

This module is part of the oracle: only tests, the smoke entry point and the
benchmark's CPU-baseline leg may use it.
"""
import numpy as np

MASK32 = np.uint64(0xFFFFFFFF)
# Multipliers and Weyl key increments of Philox4x32 (SC'11, Sec. 5).
PHILOX_M0 = np.uint64(0xD2511F53)
PHILOX_M1 = np.uint64(0xCD9E8D57)
PHILOX_W0 = np.uint64(0x9E3779B9)
PHILOX_W1 = np.uint64(0xBB67AE85)

KIND_GAUSSIAN = 0
KIND_SUBSAMPLE = 1
KIND_COUNT = 2
KIND_SRHT_SIGN = 3
KIND_SRHT_SAMPLE = 4


def philox4x32(c0, c1, c2, c3, k0, k1, rounds=10):
    """Philox4x32-R block function, vectorised over numpy arrays.

    All inputs are integer arrays (or scalars) holding 32-bit values; the
    result is four uint64 arrays holding 32-bit words.  Each round multiplies
    words 0 and 2 by the Philox constants, splits the 64-bit products into
    high and low halves, and mixes them with words 1 and 3 and the round key;
    the key is bumped by the Weyl constants between rounds.
    """
    c0, c1, c2, c3 = (np.asarray(x, dtype=np.uint64) & MASK32 for x in (c0, c1, c2, c3))
    k0 = np.asarray(k0, dtype=np.uint64) & MASK32
    k1 = np.asarray(k1, dtype=np.uint64) & MASK32
    for r in range(rounds):
        if r > 0:
            k0 = (k0 + PHILOX_W0) & MASK32
            k1 = (k1 + PHILOX_W1) & MASK32
        p0 = PHILOX_M0 * c0          # < 2^64, exact in uint64
        p1 = PHILOX_M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0) & MASK32, lo1, (hi0 ^ c3 ^ k1) & MASK32, lo0
    return c0, c1, c2, c3


def seed_key(seed):
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return seed & 0xFFFFFFFF, seed >> 32


def uniform_open01(x):
    """Map a 32-bit word to (0, 1): keep the top 23 bits and centre the cell.

    u = ((x >> 9) + 0.5) / 2^23 = (2y + 1) / 2^24 with y < 2^23 needs at most
    24 significant bits, so it is exactly representable in binary32 and
    binary64, and it is never 0 or 1, so log(u) below is always finite.
    """
    x = np.asarray(x, dtype=np.uint64)
    return ((x >> np.uint64(9)).astype(np.float64) + 0.5) * (2.0 ** -23)


def gaussian_sketch(seed, t, side, n, d, dtype=np.float64):
    """S in R^{n x d} with i.i.d. N(0, 1/d) entries (Sec. 3.4, Gaussian case).

    One Philox call per (row j, column group q) gives four words; Box-Muller
    turns (x0, x1) into columns 4q, 4q+1 and (x2, x3) into 4q+2, 4q+3.
    """
    k0, k1 = seed_key(seed)
    nq = (d + 3) // 4
    j = np.arange(n, dtype=np.uint64)[:, None]
    q = np.arange(nq, dtype=np.uint64)[None, :]
    c2 = np.uint64((side & 0xFF) | (KIND_GAUSSIAN << 8))
    x0, x1, x2, x3 = philox4x32(q + 0 * j, j + 0 * q, c2, np.uint64(t), k0, k1)
    out = np.empty((n, 4 * nq), dtype=np.float64)
    for (xa, xb, col) in ((x0, x1, 0), (x2, x3, 2)):
        ua, ub = uniform_open01(xa), uniform_open01(xb)
        rad = np.sqrt(-2.0 * np.log(ua))
        out[:, col::4] = rad * np.cos(2.0 * np.pi * ub)
        out[:, col + 1::4] = rad * np.sin(2.0 * np.pi * ub)
    return (out[:, :d] / np.sqrt(d)).astype(dtype)


def subsample_keys(seed, t, side, n, kind=KIND_SUBSAMPLE):
    """64-bit priority key of every index j < n for sampling without replacement."""
    k0, k1 = seed_key(seed)
    j = np.arange(n, dtype=np.uint64)
    c2 = np.uint64((side & 0xFF) | (kind << 8))
    x0, x1, _, _ = philox4x32(np.zeros_like(j), j, c2, np.uint64(t), k0, k1)
    return (x0 << np.uint64(32)) | x1


def subsample_indices(seed, t, side, n, d, kind=KIND_SUBSAMPLE):
    """The d sampled indices, in ascending order.

    The sampled set is the d indices with the smallest (key, index) pairs,
    i.e. a uniformly random d-subset drawn without replacement (Sec. 3.4,
    subsampling case).  Column c of S is the canonical vector of the c-th
    smallest sampled index: the order of the columns of S does not change
    S S^T, A B^T or B B^T, so the ascending order is chosen for its simpler
    parallel construction.
    """
    if not 1 <= d <= n:
        raise ValueError("subsampling needs 1 <= d <= n")
    keys = subsample_keys(seed, t, side, n, kind)
    order = np.lexsort((np.arange(n), keys))   # primary: key, secondary: index
    return np.sort(order[:d])


def subsample_sketch(seed, t, side, n, d):
    """Sparse S in R^{n x d}: S[idx[c], c] = sqrt(n/d), zero elsewhere.

    The sqrt(n/d) scale makes E[S S^T] = I (Assumption 1); unscaled canonical
    columns would give (d/n) I.
    """
    import scipy.sparse as sp
    idx = subsample_indices(seed, t, side, n, d)
    vals = np.full(d, np.sqrt(n / d))
    return sp.csc_matrix((vals, (idx, np.arange(d))), shape=(n, d))


def count_sketch_hash(seed, t, side, n, d):
    """Bucket h_j in [0, d) and sign s_j in {+1, -1} of every row j < n.

    One Philox call per row, counter (0, j, side | 2 << 8, t): the bucket is
    the high word of the 64-bit product x0 * d (a uniform draw from [0, d)
    up to a bias below 2^-32), the sign is the top bit of x1.
    """
    k0, k1 = seed_key(seed)
    j = np.arange(n, dtype=np.uint64)
    c2 = np.uint64((side & 0xFF) | (KIND_COUNT << 8))
    x0, x1, _, _ = philox4x32(np.zeros_like(j), j, c2, np.uint64(t), k0, k1)
    h = ((x0 * np.uint64(d)) >> np.uint64(32)).astype(np.int64)
    s = 1.0 - 2.0 * (x1 >> np.uint64(31)).astype(np.float64)
    return h, s


def count_sketch(seed, t, side, n, d):
    """Sparse S in R^{n x d} with one nonzero per row, S[j, h_j] = s_j.

    The count sketch that Sec. 3.4 names as applicable beyond the Gaussian
    and subsampling kinds.  (S S^T)_{jj'} = s_j s_j' [h_j = h_j'], so the
    diagonal is exactly 1 and, the signs being independent and symmetric,
    every off-diagonal entry has mean 0: E[S S^T] = I (Assumption 1).
    """
    import scipy.sparse as sp
    h, s = count_sketch_hash(seed, t, side, n, d)
    return sp.csc_matrix((s, (np.arange(n), h)), shape=(n, d))


def srht_pad(n):
    """Length N of the Hadamard transform of an n-long vector: the smallest
    power of two >= n, and at least 1024.  Any N >= n gives E[S S^T] = I;
    the paper does not fix it, and the floor keeps one transform size class
    for all short rows."""
    return max(1024, 1 << max(0, int(n - 1).bit_length()))


def srht_signs(seed, t, side, n):
    """The random signs D_jj of the SRHT, +1 or -1 by the top bit of word x0
    of counter (0, j, side | 3 << 8, t)."""
    k0, k1 = seed_key(seed)
    j = np.arange(n, dtype=np.uint64)
    c2 = np.uint64((side & 0xFF) | (KIND_SRHT_SIGN << 8))
    x0, _, _, _ = philox4x32(np.zeros_like(j), j, c2, np.uint64(t), k0, k1)
    return 1.0 - 2.0 * (x0 >> np.uint64(31)).astype(np.float64)


def hadamard_entries(a, b):
    """Entries (-1)^{popcount(a & b)} of the Sylvester-ordered Hadamard matrix
    (broadcast over integer arrays a, b)."""
    x = np.bitwise_and(np.asarray(a, dtype=np.int64), np.asarray(b, dtype=np.int64))
    parity = np.zeros(x.shape, dtype=np.int64)
    while np.any(x):
        parity ^= x & 1
        x = x >> 1
    return 1.0 - 2.0 * parity


def srht_sketch(seed, t, side, n, d):
    """Dense S in R^{n x d}: the subsampled randomised Hadamard transform.

    With N = srht_pad(n), H the N x N Sylvester Hadamard matrix (entries
    +-1), D = diag(signs) and P the N x d matrix of d canonical columns
    e_{p_c} drawn without replacement (ascending p_c),
        S = sqrt(N / d) * (first n rows of D H P) / sqrt(N),
    i.e. S[j, c] = s_j H[j, p_c] / sqrt(d).  H H^T = N I and
    E[P P^T] = (d / N) I give E[S S^T] = I (Assumption 1); with d = N = n, P
    is a permutation and S S^T = I exactly.  Sec. 3.4 names the SRHT as
    applicable and leaves it to future work; this is its standard form
    (the rows of M are padded with zeros up to N).
    """
    N = srht_pad(n)
    if not 1 <= d <= N:
        raise ValueError("the SRHT needs 1 <= d <= 2^ceil(log2 n)")
    s = srht_signs(seed, t, side, n)
    p = subsample_indices(seed, t, side, N, d, kind=KIND_SRHT_SAMPLE)
    H = hadamard_entries(np.arange(n)[:, None], p[None, :])
    return s[:, None] * H / np.sqrt(d)
