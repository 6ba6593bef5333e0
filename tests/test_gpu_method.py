"""GPU parity of whole half-iterations and of the objective against the FP64
oracle, through the context API of the C ABI."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import dsanls as O
from oracle import philox as P
from paper_2009_02845_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_02845_amd import binding
    binding.load()
    return torch, binding


def _rel(a, b):
    """Relative error: the Frobenius one, or a tenth of the largest per-row
    one (each row against its own norm, floored at 1% of the RMS row norm)
    if that is larger.  A row may thus be off by ten times the tolerance an
    assertion states for the whole array (its rounding is not averaged over
    other rows), and an error confined to a few rows (a ragged last wave,
    say) still shows."""
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    fro = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
    if b.ndim != 2 or b.shape[0] < 2:
        return fro
    rn = np.linalg.norm(b, axis=1)
    floor = max(0.01 * np.sqrt(np.mean(rn ** 2)), 1e-30)
    return max(fro, 0.1 * float(np.max(np.linalg.norm(a - b, axis=1) / np.maximum(rn, floor))))


def _ocfg(k, d, dp, sketch, solver, alpha=1.0, beta=1.0, sweeps=1, seed=0, tol=1e-4, max_sweeps=100,
          clip=False):
    return O.Config(k=k, d=d, d_prime=dp, sketch=sketch, solver=solver, alpha=alpha, beta=beta,
                    sweeps=sweeps, seed=seed, tol=tol, max_sweeps=max_sweeps, clip_upper=clip)


class Dense:
    """A dense problem living on the GPU with its oracle twin."""

    def __init__(self, env, M, U0, V0, ocfg, precision="fp32", pass_mt=False):
        torch, B = env
        self.torch, self.B = torch, B
        self.M = M.astype(np.float32)
        self.Md = torch.from_numpy(self.M).cuda()
        self.Mt = torch.from_numpy(np.ascontiguousarray(self.M.T)).cuda() if pass_mt else None
        self.U = torch.from_numpy(U0.astype(np.float32)).cuda()
        self.V = torch.from_numpy(V0.astype(np.float32)).cuda()
        m, n = M.shape
        self.ocfg = ocfg
        cfg = B.make_config(m, n, ocfg.k, ocfg.d, ocfg.d_prime, sketch=ocfg.sketch, solver=ocfg.solver,
                            precision=precision, sweeps=ocfg.sweeps, tol=ocfg.tol,
                            max_sweeps=ocfg.max_sweeps, alpha=ocfg.alpha, beta=ocfg.beta,
                            clip_upper=ocfg.clip_upper, seed=ocfg.seed)
        mat = B.dense_matrix(self.Md, self.Mt)
        self.solver = B.Solver(cfg, mat, self.U, self.V, tensors=[self.Md, self.Mt])

    def set(self, U, V):
        self.U.copy_(self.torch.from_numpy(U.astype(np.float32)))
        self.V.copy_(self.torch.from_numpy(V.astype(np.float32)))

    def get(self):
        return self.U.cpu().numpy().astype(np.float64), self.V.cpu().numpy().astype(np.float64)


def _c1(env, solver=O.SOLVER_PGD, sketch=O.SKETCH_GAUSSIAN, **kw):
    M = synth.dense_uniform(200, 150, 0, dtype=np.float64)
    U0, V0 = synth.init_factors(200, 150, 10, 0, dtype=np.float64)
    d = 150 if sketch == O.SKETCH_IDENTITY else 40
    dp = 200 if sketch == O.SKETCH_IDENTITY else 40
    ocfg = _ocfg(10, d, dp, sketch, solver, **kw)
    return M, U0, V0, ocfg


@pytest.mark.parametrize("sketch", [O.SKETCH_GAUSSIAN, O.SKETCH_SUBSAMPLE, O.SKETCH_IDENTITY])
@pytest.mark.parametrize("solver", [O.SOLVER_PGD, O.SOLVER_PROX_CD])
def test_per_update_parity_first_config(env, sketch, solver):
    M, U0, V0, ocfg = _c1(env, solver, sketch)
    prob = Dense(env, M, U0, V0, ocfg)
    M64 = M.astype(np.float32).astype(np.float64)
    U, V = U0.astype(np.float32).astype(np.float64), V0.astype(np.float32).astype(np.float64)
    for t in range(5):
        # identical inputs on both sides, one update each
        prob.set(U, V)
        prob.solver.update_U(t)
        Ug, _ = prob.get()
        Uo = O.update_U(M64, U, V, t, ocfg)
        assert _rel(Ug, Uo) < 1e-4, (t, "U")
        prob.set(Uo, V)
        prob.solver.update_V(t)
        _, Vg = prob.get()
        Vo = O.update_V(M64, Uo, V, t, ocfg)
        assert _rel(Vg, Vo) < 1e-4, (t, "V")
        assert Ug.min() >= 0 and Vg.min() >= 0
        U, V = Uo, Vo


def test_trajectory_first_config(env):
    # 200 x 150 uniform M, k = 10, Gaussian d = 40, PGD, 20 iterations
    M, U0, V0, ocfg = _c1(env)
    prob = Dense(env, M, U0, V0, ocfg)
    _, _, errs = O.run(M.astype(np.float32).astype(np.float64), U0.astype(np.float32), V0.astype(np.float32),
                       ocfg, 20)
    for t in range(20):
        prob.solver.iteration(t)
        e = prob.solver.objective()
        assert abs(e - errs[t]) / errs[t] <= 1e-3, (t, e, errs[t])


def test_intermediates_first_config(env):
    M, U0, V0, ocfg = _c1(env, O.SOLVER_PROX_CD)
    prob = Dense(env, M, U0, V0, ocfg)
    prob.solver.update_U(3)
    M64 = M.astype(np.float32).astype(np.float64)
    V = V0.astype(np.float32).astype(np.float64)
    S = P.gaussian_sketch(ocfg.seed, 3, 0, 150, 40)
    A, Bm = O.sketch_products(M64, V, S)
    G, R = O.gram_and_rhs(A, Bm)
    f = prob.solver.fetch
    assert np.max(np.abs(f(0, (40, 150)) - S.T)) < 1e-5
    assert _rel(f(1, (200, 40)), A) < 1e-5
    assert _rel(f(2, (10, 40)), Bm) < 1e-5
    assert _rel(f(3, (10, 10)), G) < 1e-5
    assert _rel(f(4, (200, 10)), R) < 1e-5


def test_objective_matches_oracle_and_planted_zero(env):
    g = np.random.default_rng(3)
    for (m, n, k) in [(200, 150, 10), (333, 129, 7), (1000, 800, 64)]:
        M = g.random((m, n))
        U, V = g.random((m, k)), g.random((n, k))
        prob = Dense(env, M, U, V, _ocfg(k, 8, 8, O.SKETCH_GAUSSIAN, O.SOLVER_PROX_CD))
        ref = O.relative_error(M.astype(np.float32).astype(np.float64), U.astype(np.float32).astype(np.float64),
                               V.astype(np.float32).astype(np.float64))
        assert abs(prob.solver.objective() - ref) / ref < 1e-5
    # exact factorisation (in FP32): residual entries are pure rounding
    U0, V0 = synth.planted_factors(300, 200, 5, 1)
    U0, V0 = U0.astype(np.float32), V0.astype(np.float32)
    M = (U0.astype(np.float64) @ V0.astype(np.float64).T)
    prob = Dense(env, M, U0, V0, _ocfg(5, 8, 8, O.SKETCH_GAUSSIAN, O.SOLVER_PROX_CD))
    assert prob.solver.objective() < 1e-6


def test_exact_anls_mode_on_planted(env):
    # identity sketch + mu = 0 + to-tolerance NNLS = exact ANLS; a noiseless
    # nonnegative rank-4 matrix is recovered to a small relative error
    U0, V0 = synth.planted_factors(60, 40, 4, 1)
    Ui, Vi = synth.init_factors(60, 40, 4, 1, dtype=np.float64)
    M = U0 @ V0.T
    ocfg = _ocfg(4, 40, 60, O.SKETCH_IDENTITY, O.SOLVER_PROX_CD, alpha=0.0, beta=0.0, sweeps=0, tol=1e-6,
                 max_sweeps=1000)
    prob = Dense(env, M, Ui, Vi, ocfg)
    for t in range(200):
        prob.solver.iteration(t)
    assert prob.solver.objective() < 2e-3


def test_passed_transpose_and_clip(env):
    M, U0, V0, ocfg = _c1(env, O.SOLVER_PROX_CD)
    ocfg.clip_upper = True
    a = Dense(env, M, U0 * 30, V0 * 30, ocfg, pass_mt=True)
    b = Dense(env, M, U0 * 30, V0 * 30, ocfg, pass_mt=False)
    for t in range(3):
        a.solver.iteration(t)
        b.solver.iteration(t)
    Ua, Va = a.get()
    Ub, Vb = b.get()
    assert np.array_equal(Ua, Ub) and np.array_equal(Va, Vb)
    ub = np.sqrt(2 * O.frobenius(M.astype(np.float32).astype(np.float64)))
    assert Ua.max() <= ub * (1 + 1e-6) and Va.max() <= ub * (1 + 1e-6)


def test_determinism_and_resume(env):
    M, U0, V0, ocfg = _c1(env, O.SOLVER_PROX_CD)
    a = Dense(env, M, U0, V0, ocfg)
    for t in range(6):
        a.solver.iteration(t)
    b = Dense(env, M, U0, V0, ocfg)
    for t in range(3):
        b.solver.iteration(t)
    Ub, Vb = b.get()
    c = Dense(env, M, Ub, Vb, ocfg)       # a fresh context resumes at t = 3
    for t in range(3, 6):
        c.solver.iteration(t)
    assert np.array_equal(a.get()[0], c.get()[0]) and np.array_equal(a.get()[1], c.get()[1])


def _sparse_problem(m, n, density, k, seed):
    g = np.random.default_rng(seed)
    Ms = sp.random(m, n, density=density, format="csr", random_state=seed, dtype=np.float64)
    Ms.data = g.lognormal(0, 1, Ms.nnz)
    Ms.sort_indices()
    U0, V0 = synth.init_factors(m, n, k, seed, dtype=np.float64)
    return Ms, U0, V0


class Sparse:
    def __init__(self, env, Ms, U0, V0, ocfg):
        torch, B = env
        self.torch = torch
        Ms = Ms.astype(np.float32).tocsr()
        Mt = Ms.T.tocsr()
        Mt.sort_indices()
        t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a.astype(dt))).cuda()
        self.arrs = [t(Ms.indptr, np.int64), t(Ms.indices, np.int32), t(Ms.data, np.float32),
                     t(Mt.indptr, np.int64), t(Mt.indices, np.int32), t(Mt.data, np.float32)]
        self.U = torch.from_numpy(U0.astype(np.float32)).cuda()
        self.V = torch.from_numpy(V0.astype(np.float32)).cuda()
        m, n = Ms.shape
        cfg = B.make_config(m, n, ocfg.k, ocfg.d, ocfg.d_prime, sketch=ocfg.sketch, solver=ocfg.solver,
                            sweeps=ocfg.sweeps, tol=ocfg.tol, max_sweeps=ocfg.max_sweeps, alpha=ocfg.alpha,
                            beta=ocfg.beta, seed=ocfg.seed)
        self.solver = B.Solver(cfg, B.csr_matrix(*self.arrs), self.U, self.V, tensors=self.arrs)

    def set(self, U, V):
        self.U.copy_(self.torch.from_numpy(U.astype(np.float32)))
        self.V.copy_(self.torch.from_numpy(V.astype(np.float32)))

    def get(self):
        return self.U.cpu().numpy().astype(np.float64), self.V.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("sketch", [O.SKETCH_SUBSAMPLE, O.SKETCH_IDENTITY])
def test_sparse_per_update_parity(env, sketch):
    m, n, k = 3000, 1200, 20
    Ms, U0, V0 = _sparse_problem(m, n, 0.01, k, 5)
    d, dp = (n, m) if sketch == O.SKETCH_IDENTITY else (120, 300)
    ocfg = _ocfg(k, d, dp, sketch, O.SOLVER_PROX_CD, alpha=0.5, beta=0.5)
    prob = Sparse(env, Ms, U0, V0, ocfg)
    M64 = Ms.astype(np.float32).astype(np.float64).tocsr()
    U, V = U0.astype(np.float32).astype(np.float64), V0.astype(np.float32).astype(np.float64)
    for t in range(3):
        prob.set(U, V)
        prob.solver.update_U(t)
        Ug, _ = prob.get()
        Uo = O.update_U(M64, U, V, t, ocfg)
        assert _rel(Ug, Uo) < 1e-4
        prob.set(Uo, V)
        prob.solver.update_V(t)
        _, Vg = prob.get()
        Vo = O.update_V(M64, Uo, V, t, ocfg)
        assert _rel(Vg, Vo) < 1e-4
        U, V = Uo, Vo
    prob.set(U, V)
    assert abs(prob.solver.objective() - O.relative_error(M64, U, V)) / O.relative_error(M64, U, V) < 1e-5


def test_sparse_run_ahead_any_call_order(env):
    # the next side's subsample and sketched rows are prepared ahead on the
    # context's second stream for (V, t) after update_U(t) and (U, t + 1)
    # after update_V(t); calls that repeat a side, skip iterations or go
    # back must wait for that work and redraw, giving the definition's
    # result every time
    m, n, k = 3000, 1200, 20
    Ms, U0, V0 = _sparse_problem(m, n, 0.01, k, 5)
    ocfg = _ocfg(k, 120, 300, O.SKETCH_SUBSAMPLE, O.SOLVER_PROX_CD, alpha=0.5, beta=0.5)
    prob = Sparse(env, Ms, U0, V0, ocfg)
    M64 = Ms.astype(np.float32).astype(np.float64).tocsr()
    U, V = U0.astype(np.float32).astype(np.float64), V0.astype(np.float32).astype(np.float64)
    for side, t in [(0, 3), (0, 3), (1, 7), (1, 3), (0, 4), (1, 4), (0, 5), (0, 9), (1, 9), (1, 9), (0, 2)]:
        prob.set(U, V)
        if side == 0:
            prob.solver.update_U(t)
            got, ref = prob.get()[0], O.update_U(M64, U, V, t, ocfg)
        else:
            prob.solver.update_V(t)
            got, ref = prob.get()[1], O.update_V(M64, U, V, t, ocfg)
        assert _rel(got, ref) < 1e-4, (side, t)


def _skewed_sparse(m, n, k, seed):
    # Zipf-like column popularity, a few fully dense rows and columns, empty
    # rows and many empty columns: sampled columns of every length (0 to m)
    # and rows of the sketched matrix longer than one lane sorts
    g = np.random.default_rng(seed)
    nnz = 6 * m
    pop = 1.0 / np.arange(1, n + 1) ** 1.1
    cols = g.choice(n, size=nnz, p=pop / pop.sum())
    rows = g.integers(0, m, size=nnz)
    dense_rows = np.repeat(g.choice(m, 3, replace=False), n)
    dense_cols = np.tile(np.arange(n), 3)
    dc = np.repeat(g.choice(n, 2, replace=False), m)
    dr = np.tile(np.arange(m), 2)
    r = np.concatenate([rows, dense_rows, dr])
    c = np.concatenate([cols, dense_cols, dc])
    Ms = sp.csr_matrix((g.lognormal(0, 1, r.size), (r, c)), shape=(m, n))
    Ms.sum_duplicates()
    Ms.sort_indices()
    empty = g.choice(m, m // 10, replace=False)
    empty_c = g.choice(n, n // 10, replace=False)
    Ms = sp.diags(np.isin(np.arange(m), empty, invert=True).astype(np.float64)) @ Ms
    Ms = Ms @ sp.diags(np.isin(np.arange(n), empty_c, invert=True).astype(np.float64))
    Ms = Ms.tocsr()
    Ms.eliminate_zeros()
    Ms.sort_indices()
    U0, V0 = synth.init_factors(m, n, k, seed, dtype=np.float64)
    return Ms, U0, V0


@pytest.mark.parametrize("m,n,d,dp", [(1500, 900, 200, 300), (3000, 900, 700, 2000), (400, 6000, 4500, 300)])
def test_sparse_subsample_skewed_parity(env, m, n, d, dp):
    # d <= 4096: sampled rows gathered through CSR(X^T), with sketched rows
    # of every length class (up to 8 entries, up to 64, up to 512, beyond:
    # the dense rows and columns give 700- and 2000-entry rows in the second
    # case); d = 4500 on the U side: the CSR stream
    k = 12
    Ms, U0, V0 = _skewed_sparse(m, n, k, 8)
    ocfg = _ocfg(k, d, dp, O.SKETCH_SUBSAMPLE, O.SOLVER_PROX_CD, alpha=0.5, beta=0.5, seed=3)
    prob = Sparse(env, Ms, U0, V0, ocfg)
    M64 = Ms.astype(np.float32).astype(np.float64).tocsr()
    U, V = U0.astype(np.float32).astype(np.float64), V0.astype(np.float32).astype(np.float64)
    for t in range(2):
        prob.set(U, V)
        prob.solver.update_U(t)
        Ug, _ = prob.get()
        Uo = O.update_U(M64, U, V, t, ocfg)
        assert _rel(Ug, Uo) < 1e-4
        prob.set(Uo, V)
        prob.solver.update_V(t)
        _, Vg = prob.get()
        Vo = O.update_V(M64, Uo, V, t, ocfg)
        assert _rel(Vg, Vo) < 1e-4
        U, V = Uo, Vo


def test_sparse_sketched_rows_skewed(env):
    # the gathered rows of A = M S equal the oracle's, slots ascending, also
    # for the near-dense rows and the empty ones
    torch, B = env
    m, n, k, d = 1500, 900, 12, 200
    Ms, U0, V0 = _skewed_sparse(m, n, k, 9)
    ocfg = _ocfg(k, d, 300, O.SKETCH_SUBSAMPLE, O.SOLVER_PROX_CD, seed=5)
    prob = Sparse(env, Ms, U0, V0, ocfg)
    prob.solver.keep_sketched_rows(True)
    prob.solver.update_U(2)
    sel = np.arange(m, dtype=np.int32)
    rp, cols, vals = prob.solver.gather_sketched_rows(torch.from_numpy(sel).cuda(), capacity=Ms.nnz)
    A = (Ms.astype(np.float32).astype(np.float64) @ P.subsample_sketch(5, 2, 0, n, d)).tocsr()
    A.sort_indices()
    got = sp.csr_matrix((vals.cpu().numpy().astype(np.float64), cols.cpu().numpy(), rp.cpu().numpy()),
                        shape=(m, d))
    assert np.array_equal(got.indptr, A.indptr) and np.array_equal(got.indices, A.indices)
    assert np.allclose(got.data, A.data, rtol=1e-6, atol=0)
    assert np.diff(A.indptr).max() > 16   # rows sorted by the workgroup path


def test_sparse_subsample_fetch_indices(env):
    Ms, U0, V0 = _sparse_problem(500, 400, 0.02, 8, 6)
    ocfg = _ocfg(8, 50, 60, O.SKETCH_SUBSAMPLE, O.SOLVER_PROX_CD, seed=17)
    prob = Sparse(env, Ms, U0, V0, ocfg)
    prob.solver.update_U(4)
    assert np.array_equal(prob.solver.fetch(0, (50,), "int32"), P.subsample_indices(17, 4, 0, 400, 50))
    prob.solver.update_V(4)
    assert np.array_equal(prob.solver.fetch(0, (60,), "int32"), P.subsample_indices(17, 4, 1, 500, 60))


@pytest.mark.parametrize("m,n,d", [(336, 208, 40), (1040, 784, 200), (528, 400, 300)])
def test_sketch_product_lds_ring_shapes(env, m, n, d):
    # m and n multiples of 16 (the contraction lengths of A = M S and
    # A' = M^T S'), so the FP32 sketch product runs on the LDS-ring kernel;
    # row tiles and d are ragged.  Intermediates and one update per side
    # against the oracle.
    k = 8
    M = synth.dense_uniform(m, n, 5, dtype=np.float64)
    U0, V0 = synth.init_factors(m, n, k, 5, dtype=np.float64)
    ocfg = _ocfg(k, d, d, O.SKETCH_GAUSSIAN, O.SOLVER_PROX_CD)
    prob = Dense(env, M, U0, V0, ocfg)
    M64 = M.astype(np.float32).astype(np.float64)
    U, V = U0.astype(np.float32).astype(np.float64), V0.astype(np.float32).astype(np.float64)
    for t in range(2):
        prob.set(U, V)
        prob.solver.update_U(t)
        S = P.gaussian_sketch(ocfg.seed, t, 0, n, d)
        A, _ = O.sketch_products(M64, V, S)
        assert _rel(prob.solver.fetch(1, (m, d)), A) < 1e-5
        Ug, _ = prob.get()
        Uo = O.update_U(M64, U, V, t, ocfg)
        assert _rel(Ug, Uo) < 1e-4
        prob.set(Uo, V)
        prob.solver.update_V(t)
        Sp = P.gaussian_sketch(ocfg.seed, t, 1, m, d)
        Ap, _ = O.sketch_products(M64.T, Uo, Sp)
        assert _rel(prob.solver.fetch(1, (n, d)), Ap) < 1e-5
        _, Vg = prob.get()
        Vo = O.update_V(M64, Uo, V, t, ocfg)
        assert _rel(Vg, Vo) < 1e-4
        U, V = Uo, Vo


@pytest.mark.parametrize("m,n,k,d", [(2000, 1200, 16, 256), (300, 180, 8, 40)])
def test_bf16_sketch_form_per_update(env, m, n, k, d):
    # planted rank-k + 1% noise, Gaussian sketch: the BF16 form matches the
    # oracle of the same form (M, S rounded to bfloat16, exact products) to
    # FP32 accuracy, and its error against the plain FP64 method is reported
    # by the bench; here it must stay small.  Neither m nor n is a multiple of
    # 32 (the BF16 copies are zero-padded to that) and 300, 180 are not of 8.
    M = synth.planted_dense(m, n, k, 2, noise_sd=0.01, noise_relative=True).astype(np.float64)
    U0, V0 = synth.init_factors(m, n, k, 2, dtype=np.float64)
    ocfg = _ocfg(k, d, d, O.SKETCH_GAUSSIAN, O.SOLVER_PROX_CD)
    ocfg.precision = "bf16"
    prob = Dense(env, M, U0, V0, ocfg, precision="bf16")
    M64 = M.astype(np.float32).astype(np.float64)
    U, V = U0.astype(np.float32).astype(np.float64), V0.astype(np.float32).astype(np.float64)
    plain = _ocfg(k, d, d, O.SKETCH_GAUSSIAN, O.SOLVER_PROX_CD)
    for t in range(3):
        prob.set(U, V)
        prob.solver.update_U(t)
        Ug, _ = prob.get()
        Uo = O.update_U(M64, U, V, t, ocfg)
        assert _rel(Ug, Uo) < 1e-4
        assert _rel(Ug, O.update_U(M64, U, V, t, plain)) < 2e-2
        prob.set(Uo, V)
        prob.solver.update_V(t)
        _, Vg = prob.get()
        Vo = O.update_V(M64, Uo, V, t, ocfg)
        assert _rel(Vg, Vo) < 1e-4
        U, V = Uo, Vo


def test_lookahead_reuse_matches_separate_calls(env):
    # update_U(t) computes the V-side sketch product too; calling update_V
    # for another t, or twice, must still give the definition's result
    M, U0, V0, ocfg = _c1(env, O.SOLVER_PROX_CD)
    prob = Dense(env, M, U0, V0, ocfg)
    M64 = M.astype(np.float32).astype(np.float64)
    U, V = U0.astype(np.float32).astype(np.float64), V0.astype(np.float32).astype(np.float64)
    prob.set(U, V)
    prob.solver.update_U(4)
    prob.solver.update_V(6)          # not the lookahead iteration
    _, Vg = prob.get()
    assert _rel(Vg, O.update_V(M64, prob.get()[0], V, 6, ocfg)) < 1e-4
    prob.set(U, V)
    prob.solver.update_V(4)          # the lookahead iteration, V-side first
    prob.solver.update_V(4)
    _, Vg2 = prob.get()
    V1 = O.update_V(M64, U, V, 4, ocfg)
    assert _rel(Vg2, O.update_V(M64, U, V1, 4, ocfg)) < 1e-4


def test_trace_env_writes_phase_totals_at_release(env, monkeypatch, capfd):
    # DSANLS_TRACE set at init: timing is on without set_timing, and releasing
    # the context writes one stderr line with the update count and the four
    # phase totals; without it nothing is written
    M, U0, V0, ocfg = _c1(env)
    monkeypatch.setenv("DSANLS_TRACE", "1")
    prob = Dense(env, M, U0, V0, ocfg)
    for t in range(3):
        prob.solver.iteration(t)
    tm = prob.solver.timing()
    assert tm["launches"] == 6 and tm["product_ms"] > 0 and tm["nnls_ms"] > 0
    capfd.readouterr()
    prob.solver.close()
    lines = [s for s in capfd.readouterr().err.splitlines() if s.startswith("[dsanls]")]
    assert len(lines) == 1 and lines[0].startswith("[dsanls] 6 updates: sketch "), lines
    assert all(f" {ph} " in lines[0] for ph in ("sketch", "product", "small", "nnls"))
    monkeypatch.setenv("DSANLS_TRACE", "0")
    quiet = Dense(env, M, U0, V0, ocfg)
    quiet.solver.iteration(0)
    assert quiet.solver.timing()["launches"] == 0
    quiet.solver.close()
    assert "[dsanls]" not in capfd.readouterr().err
