"""CSR(M^T) built on the GPU at init when the caller passes CSR(M) alone:
updates bit-identical to the ones with the caller's CSR(M^T), on a matrix
whose popular columns span many segments."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import dsanls as O
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


@pytest.mark.parametrize("sketch,d", [("subsample", 300), ("subsample", 5000), ("count", 400)])
def test_built_transpose_matches_given(env, sketch, d):
    # d = 5000 > 4096 takes the nnz stream of CSR(M^T) on the V side
    torch, B = env
    m, n, k = 30000, 6000, 20
    rp, ci, v = synth.sparse_text(m, n, 1_500_000, 4)
    Ms = sp.csr_matrix((v, ci, rp), shape=(m, n))
    Mt = Ms.T.tocsr()
    Mt.sort_indices()
    assert np.diff(Mt.indptr).max() > 4096
    U0, V0 = synth.init_factors(m, n, k, 4)
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a.astype(dt))).cuda()
    full = [t(Ms.indptr, np.int64), t(Ms.indices, np.int32), t(Ms.data, np.float32),
            t(Mt.indptr, np.int64), t(Mt.indices, np.int32), t(Mt.data, np.float32)]
    cfg = B.make_config(m, n, k, d, d, sketch=sketch, solver="prox_cd", sweeps=1, seed=1)
    Ua, Va = torch.from_numpy(U0).cuda(), torch.from_numpy(V0).cuda()
    sa = B.Solver(cfg, B.csr_matrix(*full), Ua, Va, tensors=full)
    own = B.Matrix(format=B.CSR, rowptr=full[0].data_ptr(), colidx=full[1].data_ptr(), vals=full[2].data_ptr(),
                   nnz=full[2].numel())
    Ub, Vb = torch.from_numpy(U0).cuda(), torch.from_numpy(V0).cuda()
    sb = B.Solver(cfg, own, Ub, Vb, tensors=full[:3])
    for it in range(2):
        sa.iteration(it)
        sb.iteration(it)
    torch.cuda.synchronize()
    assert torch.equal(Ua, Ub) and torch.equal(Va, Vb)
    assert sa.objective() == sb.objective()
    # and the V update against the oracle
    ocfg = O.Config(k=k, d=d, d_prime=d, sketch=O.SKETCH_SUBSAMPLE if sketch == "subsample" else O.SKETCH_COUNT,
                    solver=O.SOLVER_PROX_CD, seed=1)
    U64, V64 = Ub.cpu().numpy().astype(np.float64), Vb.cpu().numpy().astype(np.float64)
    sb.update_V(2)
    Vo = O.update_V(Ms.astype(np.float64), U64, V64, 2, ocfg, Mt=Mt.astype(np.float64))
    Vg = Vb.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(Vg - Vo) / np.linalg.norm(Vo) < 1e-4
