"""Seeded synthetic inputs shaped like the paper's workloads.

Shared by the tests, the smoke entry point and the benchmark.  This module
holds none of the factorisation method's arithmetic: it only draws matrices
(numpy PCG64, one named stream per array) so that the HIP library and the
CPU oracle can be fed identical data.

The paper evaluates on image/video matrices (dense) and text/graph matrices
(sparse, power-law); those datasets are not used here and these recipes stand
in for their shapes:
  * dense_uniform  -- M with i.i.d. uniform[0,1) entries
  * planted_dense  -- M = max(U0 V0^T + E, 0), U0, V0 entries |N(0,1)|
  * sparse_text    -- CSR with power-law row lengths, Zipf column popularity,
                      lognormal values (a text-like row block)
  * init_factors   -- U^0, V^0 with i.i.d. uniform[0,1) entries
"""
import numpy as np

_TAGS = {"M": 1, "U0": 2, "V0": 3, "noise": 4, "Uinit": 5, "Vinit": 6,
         "rows": 7, "cols": 8, "vals": 9, "perm": 10, "misc": 11}


def rng(seed, tag):
    """Independent PCG64 stream for (data seed, array name)."""
    return np.random.Generator(np.random.PCG64([int(seed), _TAGS[tag]]))


def dense_uniform(m, n, seed, dtype=np.float32):
    return rng(seed, "M").random((m, n)).astype(dtype)


def init_factors(m, n, k, seed, dtype=np.float32):
    """U^0 (m x k) and V^0 (n x k), entries uniform[0, 1)."""
    U = rng(seed, "Uinit").random((m, k)).astype(dtype)
    V = rng(seed, "Vinit").random((n, k)).astype(dtype)
    return U, V


def planted_factors(m, n, k, seed):
    U0 = np.abs(rng(seed, "U0").standard_normal((m, k)))
    V0 = np.abs(rng(seed, "V0").standard_normal((n, k)))
    return U0, V0


def planted_dense(m, n, k, seed, noise_sd=0.0, noise_relative=False,
                  dtype=np.float32, block_rows=4096):
    """M = max(U0 V0^T + E, 0) with E ~ N(0, sigma^2).

    noise_relative=True takes sigma = noise_sd * rms(U0 V0^T) ("x% noise").
    Built in row blocks so that the float64 product never exists whole.
    """
    U0, V0 = planted_factors(m, n, k, seed)
    sigma = noise_sd
    if noise_relative and noise_sd > 0:
        # rms of U0 V0^T from its Gram form: ||U0 V0^T||_F^2 = <U0^T U0, V0^T V0>
        ms = float(np.sum((U0.T @ U0) * (V0.T @ V0))) / (m * n)
        sigma = noise_sd * np.sqrt(ms)
    M = np.empty((m, n), dtype=dtype)
    g = rng(seed, "noise")
    for r0 in range(0, m, block_rows):
        r1 = min(m, r0 + block_rows)
        blk = U0[r0:r1] @ V0.T
        if sigma > 0:
            blk += sigma * g.standard_normal(blk.shape)
        M[r0:r1] = np.maximum(blk, 0.0)
    return M


def _pareto_lengths(m, target_nnz, alpha, cap, g):
    """Row lengths L = ceil(x_min u^(-1/alpha)) capped, with x_min chosen by
    bisection so that sum(L) is within 0.1% of target_nnz."""
    u = g.random(m)
    base = u ** (-1.0 / alpha)
    lo, hi = 1e-3, float(target_nnz)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        s = np.minimum(np.ceil(mid * base), cap).sum()
        if s < target_nnz:
            lo = mid
        else:
            hi = mid
        if abs(s - target_nnz) <= 1e-3 * target_nnz:
            break
    return np.minimum(np.ceil(mid * base), cap).astype(np.int64)


def sparse_text(m, n, nnz_target, seed, alpha=1.5, zipf_s=1.1, cap=None,
                dtype=np.float32):
    """Text-like CSR row block (rowptr int64, colidx int32, vals float32).

    * Row i asks for L_i entries, L ~ Pareto(alpha) (power-law document
      lengths), capped at n/10, total sum(L) ~ nnz_target.
    * Each entry's column is an i.i.d. draw from Zipf(zipf_s) over n ranks,
      mapped to columns by a seeded permutation; repeated columns within a
      row are merged (their values summed), so long rows come out a little
      shorter than L_i and the realised nnz a little below the target.
    * Values lognormal(0, 1).  Column indices are sorted within each row.
    """
    cap = cap if cap is not None else max(1, n // 10)
    L = _pareto_lengths(m, nnz_target, alpha, cap, rng(seed, "rows"))
    ranks_p = np.arange(1, n + 1, dtype=np.float64) ** (-zipf_s)
    cdf = np.cumsum(ranks_p)
    cdf /= cdf[-1]
    total = int(L.sum())
    gc = rng(seed, "cols")
    perm = rng(seed, "perm").permutation(n).astype(np.int64)
    row_of = np.repeat(np.arange(m, dtype=np.int64), L)
    col = np.empty(total, dtype=np.int64)
    chunk = 1 << 24
    for s in range(0, total, chunk):
        e = min(total, s + chunk)
        r = np.searchsorted(cdf, gc.random(e - s), side="right")
        col[s:e] = perm[np.minimum(r, n - 1)]
    vals = rng(seed, "vals").lognormal(0.0, 1.0, total)
    key = row_of * n + col
    del row_of, col
    order = np.argsort(key, kind="stable")
    key = key[order]
    vals = vals[order]
    del order
    first = np.ones(total, dtype=bool)
    first[1:] = key[1:] != key[:-1]
    grp = np.cumsum(first) - 1
    vsum = np.zeros(int(grp[-1]) + 1 if total else 0)
    np.add.at(vsum, grp, vals) if total < (1 << 22) else _segsum(vsum, grp, vals)
    ukey = key[first]
    rows = ukey // n
    cols = (ukey % n).astype(np.int32)
    rowptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=m), out=rowptr[1:])
    return rowptr, cols, vsum.astype(dtype)


def _segsum(out, grp, vals):
    # grp is sorted: bincount with weights is an exact-enough segment sum
    out[:] = np.bincount(grp, weights=vals, minlength=out.shape[0])
