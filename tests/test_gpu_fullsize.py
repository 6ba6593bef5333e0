"""GPU parity at the workloads' full sizes, in the configuration the bench
times, on sampled rows that the FP64 oracle computes one by one (the
subproblem is row-independent, eq. u_block, so the oracle's update of a set
of rows equals those rows of the full update)."""
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


def _sample(g, rows, extra, size=1500):
    return np.unique(np.concatenate([g.choice(rows, size, replace=False), extra])).astype(np.int64)


def test_sparse_text_full_size(env):
    # CSR 500000 x 200000, 1e8 nnz text-shaped, k = 100, subsampling
    # d = d' = 2000, prox-CD 1 sweep: the sampled rows include the ones with
    # the most sampled entries (the workgroup-sorted rows of A)
    torch, B = env
    m, n, k, d, nnz = 500000, 200000, 100, 2000, 100_000_000
    rp, ci, v = synth.sparse_text(m, n, nnz, 0)
    M = sp.csr_matrix((v, ci, rp), shape=(m, n))
    Mt = M.T.tocsr()
    Mt.sort_indices()
    U0, V0 = synth.init_factors(m, n, k, 0)
    dev = torch.device("cuda", 0)
    to = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a.astype(dt))).to(dev)
    keep = [to(M.indptr, np.int64), to(M.indices, np.int32), to(M.data, np.float32),
            to(Mt.indptr, np.int64), to(Mt.indices, np.int32), to(Mt.data, np.float32)]
    U, V = torch.from_numpy(U0).to(dev), torch.from_numpy(V0).to(dev)
    cfg = B.make_config(m, n, k, d, d, sketch="subsample", solver="prox_cd", sweeps=1, alpha=1.0, beta=1.0,
                        seed=0)
    s = B.Solver(cfg, B.csr_matrix(*keep), U, V, tensors=keep)
    ocfg = O.Config(k=k, d=d, d_prime=d, sketch=O.SKETCH_SUBSAMPLE, solver=O.SOLVER_PROX_CD)
    g = np.random.default_rng(1)
    M64 = M.astype(np.float64)
    U64, V64 = U0.astype(np.float64), V0.astype(np.float64)
    s.update_U(0)
    idx = P.subsample_indices(0, 0, 0, n, d)
    hits = np.diff(M[:, idx].tocsr().indptr)
    sel = _sample(g, m, np.argsort(-hits)[:40])
    Ug = U.cpu().numpy().astype(np.float64)
    assert _rel(Ug[sel], O.update_U(M64, U64, V64, 0, ocfg, rows=sel)) < 1e-4
    s.update_V(0)
    idx = P.subsample_indices(0, 0, 1, m, d)
    hits = np.diff(Mt[:, idx].tocsr().indptr)
    sel = _sample(g, n, np.argsort(-hits)[:40])
    Vg = V.cpu().numpy().astype(np.float64)
    Vo = O.update_V(M64, Ug, V64, 0, ocfg, rows=sel, Mt=Mt.astype(np.float64))
    assert _rel(Vg[sel], Vo) < 1e-4


def test_dense_planted_full_size(env):
    # dense 20000 x 10000 planted rank 64 + noise, Gaussian d = d' = 1024,
    # prox-CD 1 sweep (the sketch products are one grouped MFMA launch)
    torch, B = env
    m, n, k, d = 20000, 10000, 64, 1024
    M = synth.planted_dense(m, n, k, 0, noise_sd=0.01)
    U0, V0 = synth.init_factors(m, n, k, 0)
    dev = torch.device("cuda", 0)
    Md = torch.from_numpy(M).to(dev)
    U, V = torch.from_numpy(U0).to(dev), torch.from_numpy(V0).to(dev)
    cfg = B.make_config(m, n, k, d, d, sketch="gaussian", solver="prox_cd", sweeps=1, alpha=1.0, beta=1.0,
                        seed=0)
    s = B.Solver(cfg, B.dense_matrix(Md), U, V, tensors=[Md])
    ocfg = O.Config(k=k, d=d, d_prime=d, sketch=O.SKETCH_GAUSSIAN, solver=O.SOLVER_PROX_CD)
    g = np.random.default_rng(2)
    M64 = M.astype(np.float64)
    U64, V64 = U0.astype(np.float64), V0.astype(np.float64)
    s.update_U(0)
    sel = _sample(g, m, np.array([0, m - 1]), 400)
    Ug = U.cpu().numpy().astype(np.float64)
    assert _rel(Ug[sel], O.update_U(M64, U64, V64, 0, ocfg, rows=sel)) < 1e-4
    s.update_V(0)
    sel = _sample(g, n, np.array([0, n - 1]), 400)
    Vg = V.cpu().numpy().astype(np.float64)
    assert _rel(Vg[sel], O.update_V(M64, Ug, V64, 0, ocfg, rows=sel, Mt=M64.T)) < 1e-4


def test_dense_bf16_form_full_size(env):
    # dense 50000 x 20000 planted rank 128 + 1% noise, Gaussian d = d' = 4096,
    # BF16 sketch product (the LDS-ring kernel on zero-padded BF16 copies),
    # prox-CD 1 sweep: sampled rows against the oracle of the same form
    # (M and S rounded to bfloat16, products exact)
    torch, B = env
    m, n, k, d = 50000, 20000, 128, 4096
    M = synth.planted_dense(m, n, k, 0, noise_sd=0.01, noise_relative=True)
    U0, V0 = synth.init_factors(m, n, k, 0)
    dev = torch.device("cuda", 0)
    Md = torch.from_numpy(M).to(dev)
    U, V = torch.from_numpy(U0).to(dev), torch.from_numpy(V0).to(dev)
    cfg = B.make_config(m, n, k, d, d, sketch="gaussian", solver="prox_cd", precision="bf16", sweeps=1,
                        alpha=1.0, beta=1.0, seed=0)
    s = B.Solver(cfg, B.dense_matrix(Md), U, V, tensors=[Md])
    ocfg = O.Config(k=k, d=d, d_prime=d, sketch=O.SKETCH_GAUSSIAN, solver=O.SOLVER_PROX_CD)
    ocfg.precision = "bf16"
    g = np.random.default_rng(3)
    U64, V64 = U0.astype(np.float64), V0.astype(np.float64)
    s.update_U(0)
    sel = _sample(g, m, np.array([0, m - 1]), 200)
    Ug = U.cpu().numpy().astype(np.float64)
    assert _rel(Ug[sel], O.update_U(M, U64, V64, 0, ocfg, rows=sel)) < 1e-4
    s.update_V(0)
    sel = _sample(g, n, np.array([0, n - 1]), 200)
    Vg = V.cpu().numpy().astype(np.float64)
    assert _rel(Vg[sel], O.update_V(M, Ug, V64, 0, ocfg, rows=sel, Mt=M.T)) < 1e-4
