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


def _pareto_base(m, alpha, g):
    """Pareto(alpha) shape u^(-1/alpha) of the row lengths."""
    return g.random(m) ** (-1.0 / alpha)


def _expected_distinct(T, p, chunk=64):
    """E[#distinct columns] after T i.i.d. draws from p: sum_j 1 - (1 - p_j)^T."""
    T = np.atleast_1d(np.asarray(T, dtype=np.float64))
    lq = np.log1p(-p)
    out = np.empty_like(T)
    for s in range(0, T.size, chunk):
        out[s:s + chunk] = np.sum(-np.expm1(np.outer(T[s:s + chunk], lq)), axis=1)
    return out


def sparse_text(m, n, nnz_target, seed, alpha=1.5, zipf_s=1.1, cap=None,
                dtype=np.float32):
    """Text-like CSR row block (rowptr int64, colidx int32, vals float32).

    A bag-of-words recipe:
    * column popularity: word ranks r = 1..n with probability proportional
      to r^(-zipf_s) (Zipf), mapped to columns by a seeded permutation;
    * row i is a document of T_i tokens, each an i.i.d. word draw; repeated
      words merge into one entry whose value is the sum of the tokens'
      lognormal(0, 1) values;
    * the token counts are T_i = ceil(c * u_i^(-1/alpha)) (power-law document
      lengths), capped so that no row expects more than n/10 distinct words,
      with c set by bisection so that the expected number of distinct
      entries, sum_i sum_j 1 - (1 - p_j)^T_i, equals nnz_target.
    Column indices are sorted within each row.
    """
    cap = cap if cap is not None else max(1, n // 10)
    ranks_p = np.arange(1, n + 1, dtype=np.float64) ** (-zipf_s)
    p = ranks_p / ranks_p.sum()
    base = _pareto_base(m, alpha, rng(seed, "rows"))
    # expected distinct count as a function of T on a log grid (monotone)
    grid = np.unique(np.ceil(np.logspace(0, 8, 400)))
    dist = _expected_distinct(grid, p)
    tcap = float(np.interp(cap, dist, grid))
    def expected_nnz(c):
        T = np.minimum(np.ceil(c * base), tcap)
        return float(np.sum(np.interp(T, grid, dist))), T
    lo, hi = 1e-3, float(nnz_target)
    for _ in range(100):
        mid = np.sqrt(lo * hi)
        e, T = expected_nnz(mid)
        if e < nnz_target:
            lo = mid
        else:
            hi = mid
        if abs(e - nnz_target) <= 1e-4 * nnz_target:
            break
    L = T.astype(np.int64)
    cdf = np.cumsum(p)
    cdf /= cdf[-1]
    total = int(L.sum())
    gc = rng(seed, "cols")
    gv = rng(seed, "vals")
    perm = rng(seed, "perm").permutation(n).astype(np.int64)
    rowptr = np.zeros(m + 1, dtype=np.int64)
    cols_out, vals_out = [], []
    # process rows in chunks so the token arrays stay a few hundred MB
    starts = np.concatenate([[0], np.cumsum(L)])
    r0 = 0
    per_chunk = 1 << 25
    while r0 < m:
        r1 = int(np.searchsorted(starts, starts[r0] + per_chunk, side="right")) - 1
        r1 = max(r1, r0 + 1)
        r1 = min(r1, m)
        cnt = L[r0:r1]
        tot = int(cnt.sum())
        row_of = np.repeat(np.arange(r0, r1, dtype=np.int64), cnt)
        r = np.searchsorted(cdf, gc.random(tot), side="right")
        col = perm[np.minimum(r, n - 1)]
        v = gv.lognormal(0.0, 1.0, tot)
        key = row_of * n + col
        order = np.argsort(key, kind="stable")
        key, v = key[order], v[order]
        first = np.ones(tot, dtype=bool)
        first[1:] = key[1:] != key[:-1]
        grp = np.cumsum(first) - 1
        vsum = np.bincount(grp, weights=v)
        ukey = key[first]
        rows = ukey // n
        rowptr[r0 + 1:r1 + 1] = np.bincount(rows - r0, minlength=r1 - r0)
        cols_out.append((ukey % n).astype(np.int32))
        vals_out.append(vsum.astype(dtype))
        r0 = r1
    np.cumsum(rowptr, out=rowptr)
    del total
    return rowptr, np.concatenate(cols_out), np.concatenate(vals_out)


def mlp_init(d, k, hidden, seed, dtype=np.float32):
    """Initial warm-start network weights: uniform in +-sqrt(6 / fan_in)
    (He-uniform) for the first layer, a 100x smaller range for the output
    layer (so the initial prediction is close to the input row), zero
    biases.  W1a is d x hidden (row c holds the weights of input column c),
    W1u hidden x k, W2 k x hidden."""
    g = rng(seed, "misc")
    lim1 = np.sqrt(6.0 / (d + k))
    lim2 = 0.01 * np.sqrt(6.0 / hidden)
    return {"W1a": g.uniform(-lim1, lim1, (d, hidden)).astype(dtype),
            "W1u": g.uniform(-lim1, lim1, (hidden, k)).astype(dtype),
            "b1": np.zeros(hidden, dtype=dtype),
            "W2": g.uniform(-lim2, lim2, (k, hidden)).astype(dtype),
            "b2": np.zeros(k, dtype=dtype)}
