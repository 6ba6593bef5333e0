"""Pins of the oracle's random sketches (Sec. 3.4, Assumption 1)."""
import os

import numpy as np
import pytest
import scipy.stats

from oracle import philox
from oracle import dsanls as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _kat_rows():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append([int(w, 16) for w in line.split()])
    return rows


def test_philox_known_answers():
    rows = _kat_rows()
    assert len(rows) == 3
    for r in rows:
        out = philox.philox4x32(*r[0:4], *r[4:6])
        assert [int(x) for x in out] == r[6:10]


def test_philox_vectorised_matches_scalar():
    c0 = np.arange(17, dtype=np.uint64)
    out = philox.philox4x32(c0, 5, 7, 9, 123, 456)
    for i in range(17):
        s = philox.philox4x32(i, 5, 7, 9, 123, 456)
        assert [int(o[i]) for o in out] == [int(x) for x in s]


def test_uniform_open_interval_and_exact():
    x = np.array([0, 511, 512, 0xFFFFFFFF], dtype=np.uint64)
    u = philox.uniform_open01(x)
    assert u[0] == 0.5 * 2.0 ** -23 and u[1] == u[0]
    assert u[2] == 1.5 * 2.0 ** -23
    assert u[3] == 1.0 - 0.5 * 2.0 ** -23
    assert np.all(u.astype(np.float32).astype(np.float64) == u)


def test_gaussian_moments_and_normality():
    d = 64
    S = philox.gaussian_sketch(seed=3, t=1, side=0, n=4000, d=d)
    z = (S * np.sqrt(d)).ravel()
    N = z.size
    assert abs(z.mean()) < 4.0 / np.sqrt(N)
    assert abs(z.var() - 1.0) < 4.0 * np.sqrt(2.0 / N)
    # full distribution: Kolmogorov-Smirnov against N(0, 1)
    assert scipy.stats.kstest(z, "norm").pvalue > 1e-4
    # the two Box-Muller outputs of one pair are uncorrelated
    assert abs(np.corrcoef(z.reshape(-1, 4)[:, 0], z.reshape(-1, 4)[:, 1])[0, 1]) < 4.0 / np.sqrt(N / 4)


def test_gaussian_columns_are_philox_words():
    # S[j, 4q + 0] comes from words (x0, x1) of counter (q, j, side, t)
    seed, t, side, d = 77, 5, 1, 10
    S = philox.gaussian_sketch(seed, t, side, n=6, d=d)
    k0, k1 = philox.seed_key(seed)
    x0, x1, x2, x3 = philox.philox4x32(2, 4, side, t, k0, k1)
    ua, ub = philox.uniform_open01(x0), philox.uniform_open01(x1)
    z = np.sqrt(-2 * np.log(ua)) * np.cos(2 * np.pi * ub)
    assert np.isclose(S[4, 8], z / np.sqrt(d), rtol=0, atol=1e-15)
    assert S.shape == (6, d)


def test_distinct_streams():
    a = philox.gaussian_sketch(1, 0, 0, 50, 8)
    assert not np.allclose(a, philox.gaussian_sketch(1, 1, 0, 50, 8))   # t
    assert not np.allclose(a, philox.gaussian_sketch(1, 0, 1, 50, 8))   # side
    assert not np.allclose(a, philox.gaussian_sketch(2, 0, 0, 50, 8))   # seed
    # a block of rows is the same rows of the full sketch (global indexing)
    assert np.array_equal(philox.gaussian_sketch(1, 0, 0, 50, 8)[:20], philox.gaussian_sketch(1, 0, 0, 20, 8))


@pytest.mark.parametrize("n,d", [(10, 3), (257, 40), (1000, 1000), (64, 1)])
def test_subsample_brute_force(n, d):
    seed, t, side = 11, 4, 1
    keys = philox.subsample_keys(seed, t, side, n)
    brute = sorted(sorted(range(n), key=lambda j: (int(keys[j]), j))[:d])
    idx = philox.subsample_indices(seed, t, side, n, d)
    assert list(idx) == brute
    assert len(set(idx.tolist())) == d


def test_subsample_sketch_exact_structure():
    n, d = 300, 30
    S = philox.subsample_sketch(5, 2, 0, n, d).toarray()
    SS = S @ S.T
    diag = np.diag(SS)
    assert np.count_nonzero(diag) == d
    assert np.allclose(diag[diag > 0], n / d, rtol=0, atol=1e-12)
    assert np.count_nonzero(SS - np.diag(diag)) == 0
    # d = n: S is a permutation, S S^T = I exactly
    P = philox.subsample_sketch(5, 2, 0, 40, 40).toarray()
    assert np.array_equal(P @ P.T, np.eye(40))


@pytest.mark.parametrize("kind", [O.SKETCH_GAUSSIAN, O.SKETCH_SUBSAMPLE])
def test_assumption1_expectation_identity(kind):
    # E[S S^T] = I (Assumption 1), Monte Carlo over t
    n, d, trials = 12, 4, 3000
    acc = np.zeros((n, n))
    acc2 = np.zeros((n, n))
    for t in range(trials):
        S = O.sketch_matrix(kind, 9, t, 0, n, d)
        S = S.toarray() if hasattr(S, "toarray") else S
        P = S @ S.T
        acc += P
        acc2 += P * P
    mean = acc / trials
    sd = np.sqrt(np.maximum(acc2 / trials - mean ** 2, 1e-30) / trials)
    assert np.all(np.abs(mean - np.eye(n)) <= 5 * sd + 1e-12)


def test_bf16_rounding_matches_torch():
    import torch
    from oracle.bf16 import round_to_bf16
    g = np.random.default_rng(4)
    x = np.concatenate([g.standard_normal(20000) * 10.0 ** g.integers(-6, 6, 20000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.01171875, 3.0e38]])
    # ties: 1 + 2^-8 rounds to 1 (even), 1 + 3 * 2^-8 rounds up
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(round_to_bf16(x), ref)
    assert round_to_bf16(1.00390625) == 1.0 and round_to_bf16(1.01171875) == 1.015625


# ---- count sketch and SRHT (the further sketch kinds Sec. 3.4 names) ----

def test_count_sketch_structure_and_brute_force_product():
    n, d = 500, 37
    h, s = philox.count_sketch_hash(3, 2, 1, n, d)
    S = philox.count_sketch(3, 2, 1, n, d).toarray()
    # exactly one nonzero of +-1 per row, at the hashed bucket
    assert np.array_equal(np.count_nonzero(S, axis=1), np.ones(n))
    assert np.array_equal(S[np.arange(n), h], s) and set(np.unique(s)) == {-1.0, 1.0}
    # A = M S by adding each signed column of M into its bucket, one by one
    g = np.random.default_rng(0)
    M = g.standard_normal((6, n))
    A = np.zeros((6, d))
    for j in range(n):
        A[:, h[j]] += s[j] * M[:, j]
    assert np.allclose(O.sketch_products(M, np.zeros((n, 1)), philox.count_sketch(3, 2, 1, n, d))[0], A,
                       rtol=0, atol=1e-12)


def test_count_sketch_hash_words_and_uniformity():
    # bucket = high word of x0 * d, sign = top bit of x1, from counter (0, j, side | 2 << 8, t)
    seed, t, side, n, d = 12, 3, 0, 20000, 50
    k0, k1 = philox.seed_key(seed)
    x0, x1, _, _ = philox.philox4x32(0, 7, side | (2 << 8), t, k0, k1)
    h, s = philox.count_sketch_hash(seed, t, side, n, d)
    assert h[7] == (int(x0) * d) >> 32 and s[7] == (1.0 if int(x1) >> 31 == 0 else -1.0)
    counts = np.bincount(h, minlength=d)
    assert scipy.stats.chisquare(counts).pvalue > 1e-4
    assert abs(s.sum()) < 4 * np.sqrt(n)
    # a block of rows is the same rows of the whole sketch (global row index)
    h2, s2 = philox.count_sketch_hash(seed, t, side, 300, d)
    assert np.array_equal(h2, h[:300]) and np.array_equal(s2, s[:300])


def test_hadamard_entries_match_sylvester_construction():
    import scipy.linalg
    for N in (1, 2, 8, 64):
        a = np.arange(N)
        assert np.array_equal(philox.hadamard_entries(a[:, None], a[None, :]), scipy.linalg.hadamard(N))


def test_srht_full_width_is_orthogonal():
    # n = d = N: P is a permutation, S = D H P / sqrt(N) and S S^T = I exactly
    import scipy.linalg
    N = 1024
    S = philox.srht_sketch(5, 1, 0, N, N)
    assert np.allclose(S @ S.T, np.eye(N), rtol=0, atol=1e-12)
    p = philox.subsample_indices(5, 1, 0, N, N, kind=philox.KIND_SRHT_SAMPLE)
    assert np.array_equal(p, np.arange(N))
    D = np.diag(philox.srht_signs(5, 1, 0, N))
    assert np.allclose(S, D @ scipy.linalg.hadamard(N) / np.sqrt(N), rtol=0, atol=1e-15)
    assert philox.srht_pad(1) == 1024 and philox.srht_pad(1025) == 2048 and philox.srht_pad(4096) == 4096


def test_srht_entries_from_signs_and_sampled_columns():
    n, d = 13, 5
    S = philox.srht_sketch(9, 4, 1, n, d)
    s = philox.srht_signs(9, 4, 1, n)
    p = philox.subsample_indices(9, 4, 1, philox.srht_pad(n), d, kind=philox.KIND_SRHT_SAMPLE)
    for j in range(n):
        for c in range(d):
            par = bin(j & int(p[c])).count("1") & 1
            assert S[j, c] == s[j] * (-1.0) ** par / np.sqrt(d)


@pytest.mark.parametrize("kind", [O.SKETCH_COUNT, O.SKETCH_SRHT])
def test_assumption1_expectation_identity_further_kinds(kind):
    n, d, trials = 12, 4, 3000
    acc = np.zeros((n, n))
    acc2 = np.zeros((n, n))
    for t in range(trials):
        S = O.sketch_matrix(kind, 9, t, 0, n, d)
        S = S.toarray() if hasattr(S, "toarray") else S
        P = S @ S.T
        acc += P
        acc2 += P * P
    mean = acc / trials
    sd = np.sqrt(np.maximum(acc2 / trials - mean ** 2, 1e-30) / trials)
    assert np.all(np.abs(mean - np.eye(n)) <= 5 * sd + 1e-12)
