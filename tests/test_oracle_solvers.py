"""Pins of the oracle's subproblem solvers and products (Sec. 3.2-3.4).

Each pin checks the oracle against something other than itself: a scalar
minimiser, finite differences, a library NNLS routine, brute-force
enumeration, or a textbook special case."""
import itertools

import numpy as np
import pytest
import scipy.optimize
import scipy.sparse as sp

from oracle import dsanls as O


def _problem(rows=7, k=5, d=9, seed=0):
    g = np.random.default_rng(seed)
    A = g.standard_normal((rows, d)) + 0.5
    B = g.standard_normal((k, d))
    U = g.random((rows, k))
    return A, B, U


def _sub_objective(A, B, U, C, mu):
    """||A - U B||_F^2 + mu ||U - C||_F^2 evaluated from A and B directly."""
    return np.sum((A - U @ B) ** 2) + mu * np.sum((U - C) ** 2)


@pytest.mark.parametrize("mu", [0.0, 0.3, 5.0])
def test_prox_cd_every_coordinate_is_exact_1d_minimiser(mu):
    A, B, U0 = _problem()
    G, R = O.gram_and_rhs(A, B)
    Unew = O.prox_cd_sweep(U0.copy(), U0.copy(), G, R, mu)
    k = U0.shape[1]
    for i in range(U0.shape[0]):
        for j in range(k):
            # state seen by coordinate j: new values for l < j, old for l >= j
            state = np.concatenate([Unew[i, :j], U0[i, j:]])

            def f(x):
                u = state.copy()
                u[j] = x
                return _sub_objective(A[i:i + 1], B, u[None, :], U0[i:i + 1], mu)
            res = scipy.optimize.minimize_scalar(f, bounds=(0.0, 50.0), method="bounded",
                                                 options={"xatol": 1e-12})
            best = res.x if f(res.x) < f(0.0) else 0.0
            assert abs(Unew[i, j] - best) < 1e-6


def test_prox_cd_identity_mu0_is_hals():
    # S = I and mu = 0: one sweep is the HALS column update written in the
    # residual form u_j <- max(0, u_j + ((M V)_j - (U V^T V)_j) / (V^T V)_jj)
    g = np.random.default_rng(1)
    M = g.random((20, 15))
    U = g.random((20, 4))
    V = g.random((15, 4))
    cfg = O.Config(k=4, d=15, d_prime=20, sketch=O.SKETCH_IDENTITY, solver=O.SOLVER_PROX_CD,
                   alpha=0.0, beta=0.0, sweeps=1)
    Uo = O.update_U(M, U, V, 0, cfg)
    Uh = U.copy()
    MV, VV = M @ V, V.T @ V
    for j in range(4):
        Uh[:, j] = np.maximum(0.0, Uh[:, j] + (MV[:, j] - Uh @ VV[:, j]) / VV[j, j])
    assert np.allclose(Uo, Uh, rtol=0, atol=1e-12)


def test_prox_cd_identity_monotone_objective():
    g = np.random.default_rng(2)
    M = g.random((30, 25))
    U = g.random((30, 5))
    V = g.random((25, 5))
    cfg = O.Config(k=5, d=25, d_prime=30, sketch=O.SKETCH_IDENTITY, alpha=0.5, beta=0.0)
    f = lambda U, V: np.sum((M - U @ V.T) ** 2)
    prev = f(U, V)
    for t in range(10):
        U = O.update_U(M, U, V, t, cfg)
        cur = f(U, V)
        assert cur <= prev + 1e-12
        V = O.update_V(M, U, V, t, cfg)
        prev2 = f(U, V)
        assert prev2 <= cur + 1e-12
        prev = prev2


def _brute_force_nnls(Q, q):
    """Unique minimiser of 1/2 u Q u^T - q u^T over u >= 0 by enumerating all
    2^k passive sets (Q positive definite)."""
    k = Q.shape[0]
    for mask in itertools.product([False, True], repeat=k):
        P = np.array(mask)
        u = np.zeros(k)
        if P.any():
            u[P] = np.linalg.solve(Q[np.ix_(P, P)], q[P])
        if np.any(u[P] < -1e-12):
            continue
        g = u @ Q - q
        if np.all(g[~P] >= -1e-10):
            return np.maximum(u, 0.0)
    raise AssertionError("no KKT point found")


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_to_tol_matches_active_set_enumeration(k):
    A, B, U0 = _problem(rows=6, k=k, d=12, seed=k)
    G, R = O.gram_and_rhs(A, B)
    mu = 0.7
    U, used = O.prox_cd_solve(U0, U0, G, R, mu, sweeps=0, tol=1e-12, max_sweeps=5000)
    Q = G + mu * np.eye(k)
    for i in range(U0.shape[0]):
        ub = _brute_force_nnls(Q, R[i] + mu * U0[i])
        assert np.allclose(U[i], ub, rtol=0, atol=1e-8)
    assert np.all(used >= 0)


@pytest.mark.parametrize("k,mu", [(10, 0.5), (30, 2.0), (8, 0.0)])
def test_to_tol_matches_lawson_hanson(k, mu):
    # scipy.optimize.nnls on [B^T; sqrt(mu) I] u = [a; sqrt(mu) c]
    A, B, U0 = _problem(rows=5, k=k, d=3 * k, seed=10 + k)
    G, R = O.gram_and_rhs(A, B)
    U, _ = O.prox_cd_solve(U0, U0, G, R, mu, sweeps=0, tol=1e-13, max_sweeps=20000)
    for i in range(5):
        Ab = np.vstack([B.T, np.sqrt(mu) * np.eye(k)])
        bb = np.concatenate([A[i], np.sqrt(mu) * U0[i]])
        ref, _ = scipy.optimize.nnls(Ab, bb, maxiter=5000)
        assert np.allclose(U[i], ref, rtol=0, atol=1e-7)
        assert O.kkt_residual(U[i:i + 1], U0[i:i + 1], G, R[i:i + 1], mu)[0] <= 1e-13


def test_kkt_residual_zero_only_at_solution():
    A, B, U0 = _problem(rows=3, k=6, d=15, seed=4)
    G, R = O.gram_and_rhs(A, B)
    mu = 1.0
    Us = np.empty_like(U0)
    for i in range(3):
        Ab = np.vstack([B.T, np.eye(6)])
        Us[i], _ = scipy.optimize.nnls(Ab, np.concatenate([A[i], U0[i]]))
    assert np.all(O.kkt_residual(Us, U0, G, R, mu) < 1e-9)
    assert np.all(O.kkt_residual(Us + 0.01, U0, G, R, mu) > 1e-4)


def test_pgd_direction_is_finite_difference_gradient():
    A, B, U = _problem(rows=4, k=3, d=8, seed=5)
    U = U + 1.0                   # interior: no projection
    G, R = O.gram_and_rhs(A, B)
    eta = 1e-3
    h = 1e-6
    gfd = np.zeros_like(U)
    for i in range(U.shape[0]):
        for j in range(U.shape[1]):
            Up, Um = U.copy(), U.copy()
            Up[i, j] += h
            Um[i, j] -= h
            gfd[i, j] = (np.sum((A - Up @ B) ** 2) - np.sum((A - Um @ B) ** 2)) / (2 * h)
    assert np.allclose(O.pgd_step(U, G, R, eta), np.maximum(U - eta * gfd, 0), rtol=0, atol=1e-8)


def test_pgd_fixed_point_and_descent_identity_sketch():
    g = np.random.default_rng(6)
    M = g.random((12, 9))
    V = g.random((9, 3))
    G, R = V.T @ V, M @ V
    Us = np.array([scipy.optimize.nnls(V, M[i])[0] for i in range(12)])
    eta = O.pgd_step_size(G, 0.0)
    assert np.allclose(O.pgd_step(Us, G, R, eta), Us, rtol=0, atol=1e-10)
    assert np.max(np.sum(np.abs(G), axis=0)) >= np.max(np.linalg.eigvalsh(G)) - 1e-12
    U = g.random((12, 3))
    f = lambda U: np.sum((M - U @ V.T) ** 2)
    for _ in range(20):
        Un = O.pgd_step(U, G, R, eta)
        assert f(Un) <= f(U) + 1e-12
        U = Un


def test_identity_sketch_products():
    g = np.random.default_rng(7)
    M = g.random((8, 6))
    V = g.random((6, 2))
    S = O.sketch_matrix(O.SKETCH_IDENTITY, 0, 0, 0, 6, 6)
    A, B = O.sketch_products(M, V, S)
    assert np.allclose(A, M) and np.allclose(B, V.T)


def test_sparse_and_dense_paths_agree():
    g = np.random.default_rng(8)
    Md = g.random((40, 30)) * (g.random((40, 30)) < 0.2)
    Ms = sp.csr_matrix(Md)
    U = g.random((40, 4))
    V = g.random((30, 4))
    for kind in (O.SKETCH_SUBSAMPLE, O.SKETCH_GAUSSIAN):
        cfg = O.Config(k=4, d=10, d_prime=12, sketch=kind, seed=3)
        assert np.allclose(O.update_U(Md, U, V, 2, cfg), O.update_U(Ms, U, V, 2, cfg), atol=1e-12)
        assert np.allclose(O.update_V(Md, U, V, 2, cfg), O.update_V(Ms, U, V, 2, cfg), atol=1e-12)
    assert abs(O.relative_error(Md, U, V) - O.relative_error(Ms, U, V)) < 1e-12


def test_row_subset_update_is_row_independent():
    g = np.random.default_rng(9)
    M = g.random((25, 20))
    U = g.random((25, 3))
    V = g.random((20, 3))
    cfg = O.Config(k=3, d=8, d_prime=9, seed=1)
    full = O.update_U(M, U, V, 4, cfg)
    rows = np.array([0, 7, 24])
    assert np.allclose(O.update_U(M, U, V, 4, cfg, rows=rows), full[rows], atol=1e-13)


def test_objective_special_values():
    g = np.random.default_rng(10)
    U = g.random((9, 2))
    V = g.random((7, 2))
    M = U @ V.T
    assert O.relative_error(M, U, V) < 1e-15
    assert abs(O.relative_error(M, 0 * U, V) - 1.0) < 1e-15
    Ms = sp.csr_matrix(M * (M > 0.5))
    Md = Ms.toarray()
    assert abs(O.relative_error(Ms, U, V) - np.sqrt(np.sum((Md - U @ V.T) ** 2) / np.sum(Md ** 2))) < 1e-12


@pytest.mark.parametrize("kind", [O.SKETCH_GAUSSIAN, O.SKETCH_SUBSAMPLE])
def test_sketched_gradient_is_unbiased(kind):
    # E[2 (U V^T - M) S S^T V] = 2 (U V^T - M) V  (the unbiasedness lemma)
    g = np.random.default_rng(11)
    m, n, k, d = 5, 16, 2, 4
    M = g.random((m, n))
    U = g.random((m, k))
    V = g.random((n, k))
    trials = 4000
    acc = np.zeros((m, k))
    acc2 = np.zeros((m, k))
    for t in range(trials):
        S = O.sketch_matrix(kind, 21, t, 0, n, d)
        A, B = O.sketch_products(M, V, S)
        G, R = O.gram_and_rhs(A, B)
        gt = 2 * (U @ G - R)
        acc += gt
        acc2 += gt * gt
    mean = acc / trials
    sd = np.sqrt((acc2 / trials - mean ** 2) / trials)
    exact = 2 * (U @ V.T - M) @ V
    assert np.all(np.abs(mean - exact) <= 5 * sd)


@pytest.mark.parametrize("kind", [O.SKETCH_COUNT, O.SKETCH_SRHT])
def test_sketched_gradient_is_unbiased_further_kinds(kind):
    g = np.random.default_rng(12)
    m, n, k, d = 5, 13, 2, 4
    M = g.random((m, n))
    U = g.random((m, k))
    V = g.random((n, k))
    trials = 4000
    acc = np.zeros((m, k))
    acc2 = np.zeros((m, k))
    for t in range(trials):
        S = O.sketch_matrix(kind, 22, t, 0, n, d)
        A, B = O.sketch_products(M, V, S)
        G, R = O.gram_and_rhs(A, B)
        gt = 2 * (U @ G - R)
        acc += gt
        acc2 += gt * gt
    mean = acc / trials
    sd = np.sqrt((acc2 / trials - mean ** 2) / trials)
    exact = 2 * (U @ V.T - M) @ V
    assert np.all(np.abs(mean - exact) <= 5 * sd)


def test_prox_cd_zero_gram_column_without_mu_is_set_to_zero():
    # a coordinate whose column of B is zero does not enter the objective
    # when mu = 0; the sweep sets it to 0 (one of its minimisers) and the
    # other coordinates still take their exact 1-D minimisers
    A, B, U0 = _problem(rows=4, k=4, d=9, seed=13)
    B[2] = 0.0
    G, R = O.gram_and_rhs(A, B)
    U = O.prox_cd_sweep(U0.copy(), U0.copy(), G, R, 0.0)
    assert np.all(U[:, 2] == 0.0)
    for i in range(4):
        for j in (0, 1, 3):
            state = np.concatenate([U[i, :j], U0[i, j:]])
            state[2] = U[i, 2] if j > 2 else U0[i, 2]
            num = R[i, j] - sum(G[l, j] * state[l] for l in range(4) if l != j)
            assert abs(U[i, j] - max(num / G[j, j], 0.0)) < 1e-12


def test_prox_cd_clip_and_nan_propagation():
    A, B, U0 = _problem(rows=3, k=3, d=7, seed=14)
    G, R = O.gram_and_rhs(A, B)
    U = O.prox_cd_sweep(U0.copy(), U0.copy(), G, R, 0.5, upper=0.05)
    assert np.all(U <= 0.05) and np.all(U >= 0)
    # a NaN right-hand side is not projected to 0: it stays NaN in its row
    Rn = R.copy()
    Rn[1, 0] = np.nan
    Un = O.prox_cd_sweep(U0.copy(), U0.copy(), G, Rn, 0.5)
    assert np.isnan(Un[1, 0]) and np.all(np.isfinite(Un[[0, 2]]))
