"""The proximal weight mu_t = alpha + beta t is chosen as the paper does
(Sec. 5.2: alpha, beta in {0.1, 1, 10}, the best per data set): on the
oracle, for the 200 x 150 parity case, the (alpha, beta) the benchmark uses
is the grid's best after its 20 iterations, for each solver."""
import os
import sys

import numpy as np
import pytest

from oracle import dsanls as O
from paper_2009_02845_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GRID = (0.1, 1.0, 10.0)


def _grid(solver):
    M = synth.dense_uniform(200, 150, 0).astype(np.float64)
    U0, V0 = synth.init_factors(200, 150, 10, 0)
    out = {}
    for a in GRID:
        for b in GRID:
            cfg = O.Config(k=10, d=40, d_prime=40, sketch=O.SKETCH_GAUSSIAN, solver=solver, alpha=a, beta=b, seed=0)
            out[(a, b)] = O.run(M, U0, V0, cfg, 20)[2][-1]
    return out


@pytest.mark.parametrize("solver", [O.SOLVER_PGD, O.SOLVER_PROX_CD])
def test_bench_uses_the_grid_winner_on_the_parity_case(solver):
    sys.path.insert(0, ROOT)
    import bench
    res = _grid(solver)
    best = min(res, key=res.get)
    if solver == O.SOLVER_PGD:
        w = bench.WORKLOADS["dense-200x150"]
    else:
        w = [c for c in bench.WORKLOADS["pgd-vs-cd"]["cases"] if c["name"] == "dense-200x150"][0]
        w = dict(w, **w.get("prox_cd", {}))
    assert (w.get("alpha", 1.0), w.get("beta", 1.0)) == best, (best, res[best])
    # every grid point still decreases the objective from the start
    M = synth.dense_uniform(200, 150, 0).astype(np.float64)
    U0, V0 = synth.init_factors(200, 150, 10, 0)
    start = O.relative_error(M, U0.astype(np.float64), V0.astype(np.float64))
    assert all(v < start for v in res.values())
