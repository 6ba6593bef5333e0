"""GPU parity of the count sketch and the SRHT (the further sketch kinds of
Sec. 3.4's last paragraph) against the FP64 oracle: the sketch products,
whole updates on dense and CSR input, a node's share, and the objective
trajectory."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import dsanls as O
from paper_2009_02845_amd import synth

pytestmark = pytest.mark.gpu

KIND = {"count": O.SKETCH_COUNT, "srht": O.SKETCH_SRHT}


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


def _dense(env, M, U0, V0, sketch, k, d, dp, **kw):
    torch, B = env
    Md = torch.from_numpy(np.ascontiguousarray(M.astype(np.float32))).cuda()
    U = torch.from_numpy(np.ascontiguousarray(U0.astype(np.float32))).cuda()
    V = torch.from_numpy(np.ascontiguousarray(V0.astype(np.float32))).cuda()
    m, n = M.shape
    cfg = B.make_config(m, n, k, d, dp, sketch=sketch, solver=kw.pop("solver", "prox_cd"), seed=5, **kw)
    return B.Solver(cfg, B.dense_matrix(Md), U, V, tensors=[Md]), U, V


@pytest.mark.parametrize("sketch", ["count", "srht"])
@pytest.mark.parametrize("m,n,k,d,dp", [(200, 150, 10, 40, 40), (333, 257, 7, 29, 61), (64, 1500, 33, 300, 17)])
def test_dense_products_and_updates_match_oracle(env, sketch, m, n, k, d, dp):
    # A = M S, B = V^T S, G, R and the prox-CD update of each side from the
    # oracle's state (shapes with ragged tails, d above and below k)
    M = synth.dense_uniform(m, n, 1).astype(np.float64)
    U0, V0 = (x.astype(np.float64) for x in synth.init_factors(m, n, k, 1))
    s, U, V = _dense(env, M, U0, V0, sketch, k, d, dp)
    ocfg = O.Config(k=k, d=d, d_prime=dp, sketch=KIND[sketch], solver=O.SOLVER_PROX_CD, seed=5)
    Mf = M.astype(np.float32).astype(np.float64)
    Uf, Vf = U0.astype(np.float32).astype(np.float64), V0.astype(np.float32).astype(np.float64)
    for t in range(3):
        s.update_U(t)
        S = O.sketch_matrix(KIND[sketch], 5, t, 0, n, d)
        A, Bm = O.sketch_products(Mf, Vf, S)
        A = A.toarray() if sp.issparse(A) else A
        G, R = O.gram_and_rhs(A, Bm)
        assert _rel(s.fetch(1, (m, d)), A) < 1e-5
        assert _rel(s.fetch(2, (k, d)), Bm) < 1e-5
        assert _rel(s.fetch(3, (k, k)), G) < 1e-5
        assert _rel(s.fetch(4, (m, k)), R) < 1e-5
        Uo = O.update_U(Mf, Uf, Vf, t, ocfg)
        Ug = U.cpu().numpy().astype(np.float64)
        assert _rel(Ug, Uo) < 1e-4
        s.update_V(t)
        Vo = O.update_V(Mf, Ug, Vf, t, ocfg)
        Vg = V.cpu().numpy().astype(np.float64)
        assert _rel(Vg, Vo) < 1e-4
        # next update from the GPU's state on both sides
        Uf, Vf = Ug, Vg


@pytest.mark.parametrize("sketch", ["count", "srht"])
def test_dense_trajectory_matches_oracle(env, sketch):
    # 20 iterations of the parity case: objective within 1e-3 at every t
    m, n, k, d = 200, 150, 10, 40
    M = synth.dense_uniform(m, n, 0).astype(np.float64)
    U0, V0 = (x.astype(np.float64) for x in synth.init_factors(m, n, k, 0))
    s, U, V = _dense(env, M, U0, V0, sketch, k, d, d)
    ocfg = O.Config(k=k, d=d, d_prime=d, sketch=KIND[sketch], solver=O.SOLVER_PROX_CD, seed=5)
    Mf = M.astype(np.float32).astype(np.float64)
    _, _, errs = O.run(Mf, U0.astype(np.float32), V0.astype(np.float32), ocfg, 20)
    for t in range(20):
        s.iteration(t)
        assert abs(s.objective() - errs[t]) / errs[t] < 1e-3


def test_srht_longest_transform(env):
    # n = 20000 columns: N = 32768, the largest transform (1024 threads, 32
    # values each); a few rows, both the product and the update
    m, n, k, d = 96, 20000, 16, 512
    M = synth.dense_uniform(m, n, 2).astype(np.float64)
    U0, V0 = (x.astype(np.float64) for x in synth.init_factors(m, n, k, 2))
    s, U, V = _dense(env, M, U0, V0, "srht", k, d, 64)
    s.update_U(4)
    S = O.sketch_matrix(O.SKETCH_SRHT, 5, 4, 0, n, d)
    Mf = M.astype(np.float32).astype(np.float64)
    Vf = V0.astype(np.float32).astype(np.float64)
    assert _rel(s.fetch(1, (m, d)), Mf @ S) < 1e-5
    ocfg = O.Config(k=k, d=d, d_prime=64, sketch=O.SKETCH_SRHT, solver=O.SOLVER_PROX_CD, seed=5)
    Uo = O.update_U(Mf, U0.astype(np.float32).astype(np.float64), Vf, 4, ocfg)
    assert _rel(U.cpu().numpy().astype(np.float64), Uo) < 1e-4


def _csr(env, Ms, U0, V0, k, d, dp, **kw):
    torch, B = env
    Ms = Ms.tocsr()
    Ms.sort_indices()
    Mt = Ms.T.tocsr()
    Mt.sort_indices()
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a.astype(dt))).cuda()
    arrs = [t(Ms.indptr, np.int64), t(Ms.indices, np.int32), t(Ms.data, np.float32),
            t(Mt.indptr, np.int64), t(Mt.indices, np.int32), t(Mt.data, np.float32)]
    U, V = torch.from_numpy(np.ascontiguousarray(U0)).cuda(), torch.from_numpy(np.ascontiguousarray(V0)).cuda()
    cfg = B.make_config(Ms.shape[0], Ms.shape[1], k, d, dp, sketch="count", solver="prox_cd", seed=5, **kw)
    return B.Solver(cfg, B.csr_matrix(*arrs), U, V, tensors=arrs), U, V


@pytest.mark.parametrize("k", [10, 64, 100])
def test_csr_count_sketch_updates_match_oracle(env, k):
    # the nnz stream folds M_ij s_j B^T[h_j, :] into R (skewed rows, some
    # longer than one 4096-entry segment)
    torch, B = env
    m, n, d = 1200, 9000, 300
    g = np.random.default_rng(6)
    lens = np.minimum((g.pareto(1.5, m) + 1) * 8, n).astype(np.int64)
    lens[[3, 700]] = [6000, 8500]
    rows = np.repeat(np.arange(m), lens)
    cols = np.concatenate([g.choice(n, L, replace=False) for L in lens])
    Ms = sp.csr_matrix((g.lognormal(0, 1, len(rows)).astype(np.float32), (rows, cols)), shape=(m, n))
    U0, V0 = synth.init_factors(m, n, k, 6)
    s, U, V = _csr(env, Ms, U0, V0, k, d, d)
    ocfg = O.Config(k=k, d=d, d_prime=d, sketch=O.SKETCH_COUNT, solver=O.SOLVER_PROX_CD, seed=5)
    M64 = Ms.astype(np.float64)
    U64, V64 = U0.astype(np.float64), V0.astype(np.float64)
    s.update_U(1)
    S = O.sketch_matrix(O.SKETCH_COUNT, 5, 1, 0, n, d)
    A, Bm = O.sketch_products(M64, V64, S)
    _, R = O.gram_and_rhs(A, Bm)
    assert _rel(s.fetch(4, (m, k)), R) < 1e-5
    Ug = U.cpu().numpy().astype(np.float64)
    assert _rel(Ug, O.update_U(M64, U64, V64, 1, ocfg)) < 1e-4
    s.update_V(1)
    assert _rel(V.cpu().numpy().astype(np.float64), O.update_V(M64, Ug, V64, 1, ocfg)) < 1e-4


@pytest.mark.parametrize("sketch", ["count", "srht"])
def test_row_block_share_reproduces_the_whole(env, sketch):
    # sketch rows drawn at global indices: a row block (all columns) updates
    # its rows exactly as the whole matrix does; a column block its V rows
    m, n, k, d = 300, 240, 8, 36
    M = synth.dense_uniform(m, n, 7)
    U0, V0 = synth.init_factors(m, n, k, 7)
    whole, Uw, Vw = _dense(env, M, U0, V0, sketch, k, d, d)
    whole.update_U(2)
    whole.update_V(2)
    Uwhole, Vwhole = Uw.cpu().numpy(), Vw.cpu().numpy()
    r0, r1 = 120, 300
    blk, Ub, _ = _dense(env, M[r0:r1], U0[r0:r1], V0, sketch, k, d, d, row_offset=r0, m_global=m)
    blk.update_U(2)
    assert _rel(Ub.cpu().numpy(), Uwhole[r0:r1]) < 1e-5
    c0, c1 = 100, 240
    blk, _, Vb = _dense(env, M[:, c0:c1], Uwhole, V0[c0:c1], sketch, k, d, d, col_offset=c0, n_global=n)
    blk.update_V(2)
    assert _rel(Vb.cpu().numpy(), Vwhole[c0:c1]) < 1e-5


def test_limits_are_reported(env):
    torch, B = env
    M = torch.zeros((10, 40000), device="cuda")
    U, V = torch.zeros((10, 4), device="cuda"), torch.zeros((40000, 4), device="cuda")
    with pytest.raises(B.DsanlsError) as e:
        B.Solver(B.make_config(10, 40000, 4, 8, 8, sketch="srht"), B.dense_matrix(M), U, V, tensors=[M])
    assert e.value.status_name == "UNSUPPORTED"
    with pytest.raises(B.DsanlsError) as e:
        B.Solver(B.make_config(10, 40000, 4, 8, 8, sketch="count"), B.dense_matrix(M), U, V, tensors=[M])
    assert e.value.status_name == "UNSUPPORTED"
