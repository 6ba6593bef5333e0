"""The allocation-free NNLS entry point (static device scratch) gives the
same results as the workspace entry point, on two calls in a row with the
second one smaller (the scratch keeps the first call's contents)."""
import numpy as np
import pytest

from oracle import dsanls as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2009_02845_amd import binding
    binding.load()
    return torch, binding


def _problem(rows, k, d, seed):
    g = np.random.default_rng(seed)
    B = g.standard_normal((k, d))
    A = g.standard_normal((rows, d)) + 0.3
    G, R = O.gram_and_rhs(A, B)
    U0 = g.random((rows, k))
    return G, R, U0


@pytest.mark.parametrize("sweeps", [1, 0])
def test_noalloc_matches_workspace_entry_point(env, sweeps):
    torch, Bd = env
    assert 0 < Bd.load().dsanls_nnls_noalloc_scratch_bytes() <= 1 << 22
    for rows, k, d, mu in ((5000, 100, 150, 0.7), (777, 33, 50, 1.3)):
        G, R, U0 = _problem(rows, k, d, rows + sweeps)
        t = lambda x: torch.from_numpy(np.ascontiguousarray(x.astype(np.float32))).cuda()
        Gd, Rd = t(G), t(R)
        Ua, Ub = t(U0), t(U0)
        ua = Bd.nnls_prox_cd(Gd, Rd, Ua, Ua, mu, sweeps=sweeps, tol=1e-5, max_sweeps=200, want_sweeps=True)
        ub = Bd.nnls_prox_cd_noalloc(Gd, Rd, Ub, Ub, mu, sweeps=sweeps, tol=1e-5, max_sweeps=200,
                                     want_sweeps=True)
        torch.cuda.synchronize()
        # same kernels on the same inputs: identical bits, identical sweep counts
        assert torch.equal(Ua, Ub)
        assert torch.equal(ua, ub)
        # and the oracle's update within the FP32 bar
        Uo, _ = O.prox_cd_solve(U0.astype(np.float32).astype(np.float64), U0.astype(np.float32).astype(np.float64),
                                G.astype(np.float32).astype(np.float64), R.astype(np.float32).astype(np.float64),
                                mu, sweeps, tol=1e-5 if sweeps == 0 else 1e-4, max_sweeps=200)
        err = np.linalg.norm(Ub.cpu().numpy() - Uo) / np.linalg.norm(Uo)
        assert err < (1e-3 if sweeps == 0 else 1e-4)


def test_noalloc_rejects_ranks_beyond_the_scratch(env):
    torch, Bd = env
    G = torch.zeros((200, 200), device="cuda")
    R = torch.zeros((4, 200), device="cuda")
    U = torch.zeros((4, 200), device="cuda")
    with pytest.raises(Bd.DsanlsError) as e:
        Bd.nnls_prox_cd_noalloc(G, R, U, U, 1.0)
    assert e.value.status_name == "UNSUPPORTED"
