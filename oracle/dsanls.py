"""FP64 CPU oracle of sketched ANLS / DSANLS at one node (test infrastructure).

This is a plain, slow, deliberately unoptimised restatement of the method of
"Fast and Secure Distributed Nonnegative Matrix Factorization" (arXiv
2009.02845) with N = 1 node.  It exists only to check the HIP library: tests,
the smoke entry point and the benchmark's CPU-baseline leg may import it; the
product path never does.  It shares no code with the library.

The method (Sec. 3, Alg. 2 with N = 1):
  for t = 0 .. T-1:
    S^t  = random n x d sketch                      (Sec. 3.4)
    A^t  = M S^t,  B^t = V^T S^t                    (eq. def_A_B)
    U    <- one step on  min_{U>=0} ||A^t - U B^t||_F^2   (Sec. 3.5)
    S'^t = random m x d' sketch
    A'^t = M^T S'^t,  B'^t = U^T S'^t               (U is the new U, Alg. 1)
    V    <- one step on  min_{V>=0} ||A'^t - V B'^t||_F^2
The step is either one projected-gradient step (eq. gradient_descent) or one
sweep of proximal coordinate descent (eq. reg_sub, eq. entry_sol, Alg. 3).

Readings where the paper is silent or inconsistent are documented inline:
  * mu_t = alpha + beta * t with t counted from 0 (Sec. 5.2 setup).
  * The V-update uses the freshly updated U (Alg. 1), not U^t.
  * The PGD step size is eta_t = 1 / (2 (L_t + mu_t)) with L_t the largest
    absolute column sum of G = B B^T (a Gershgorin bound on its top
    eigenvalue); the paper only asks for a diminishing step.
  * More than one sweep, or sweeping to a tolerance, keeps the proximal
    centre at U^t; later sweeps use the current values of all coordinates.
"""
from dataclasses import dataclass, field
import math

import numpy as np
import scipy.sparse as sp

from . import bf16 as _bf16
from . import philox

SKETCH_GAUSSIAN = "gaussian"
SKETCH_SUBSAMPLE = "subsample"
SKETCH_IDENTITY = "identity"
SKETCH_COUNT = "count"
SKETCH_SRHT = "srht"
SOLVER_PROX_CD = "prox_cd"
SOLVER_PGD = "pgd"


@dataclass
class Config:
    k: int
    d: int
    d_prime: int
    sketch: str = SKETCH_GAUSSIAN
    solver: str = SOLVER_PROX_CD
    alpha: float = 1.0
    beta: float = 1.0
    sweeps: int = 1            # prox-CD sweeps per update; 0 means "to tolerance"
    tol: float = 1e-4          # KKT tolerance for sweeps == 0
    max_sweeps: int = 100
    clip_upper: bool = False   # optional box of eq. extra_con
    seed: int = 0
    precision: str = "fp32"    # "bf16": M and S rounded to bfloat16 for A = M S


def mu_t(cfg, t):
    """Proximal weight mu_t = alpha + beta t (Sec. 5.2), growing without bound."""
    return cfg.alpha + cfg.beta * t


# ----------------------------------------------------------------------------
# Sketch matrices (Sec. 3.4)
# ----------------------------------------------------------------------------

def sketch_matrix(kind, seed, t, side, n, d):
    """The n x d sketch for one half-iteration (dense ndarray or scipy sparse)."""
    if kind == SKETCH_GAUSSIAN:
        return philox.gaussian_sketch(seed, t, side, n, d)
    if kind == SKETCH_SUBSAMPLE:
        return philox.subsample_sketch(seed, t, side, n, d)
    if kind == SKETCH_COUNT:
        return philox.count_sketch(seed, t, side, n, d)
    if kind == SKETCH_SRHT:
        return philox.srht_sketch(seed, t, side, n, d)
    if kind == SKETCH_IDENTITY:
        if d != n:
            raise ValueError("identity sketch needs d == n")
        return sp.identity(n, format="csc", dtype=np.float64)
    raise ValueError(kind)


def _dense(x):
    return x.toarray() if sp.issparse(x) else np.asarray(x)


# ----------------------------------------------------------------------------
# Sketch products (eq. def_A_B) and the quantities of the gradient
# ----------------------------------------------------------------------------

def sketch_products(Mx, W, S):
    """A = Mx S (rows x d) and B = W^T S (k x d).

    For the U-subproblem Mx = M and W = V; for the V-subproblem Mx = M^T and
    W = U (Alg. 2).  Mx may be dense or scipy-sparse, S dense or sparse.
    """
    A = Mx @ S
    B = (S.T @ W).T if sp.issparse(S) else W.T @ S
    return A, _dense(B)


def gram_and_rhs(A, B):
    """G = B B^T (k x k) and R = A B^T (rows x k): the two products of the
    sketched gradient 2[U B B^T - A B^T] (eq. gradient_descent)."""
    G = B @ B.T
    R = A @ B.T
    return _dense(G), _dense(R)


# ----------------------------------------------------------------------------
# Subproblem solvers (Sec. 3.5)
# ----------------------------------------------------------------------------

def prox_cd_sweep(U, C, G, R, mu, upper=None):
    """One sweep of proximal coordinate descent (Alg. 3), in place on U.

    Every row u of U has its own quadratic (eq. reg_sub, halved)
        f(u) = 1/2 u Q u^T - q u^T,   Q = G + mu I,   q = r + mu c,
    with c the row of the proximal centre C (= U^t).  The coordinates are
    visited in order j = 0 .. k-1 and each is set to the exact minimiser of
    f over u_j >= 0 with the other coordinates held at their current values
    (eq. entry_sol): f restricted to u_j is a parabola of curvature Q_jj
    whose slope at the current point is h_j = (u Q - q)_j, so the minimiser
    is the Newton point u_j - h_j / Q_jj projected onto [0, upper].  The
    slopes of all coordinates are kept in h for the whole block of rows: when
    u_j moves by delta, h gains delta times row j of Q, so coordinate j + 1
    sees the values already updated in this sweep (Gauss-Seidel order).

    Where the paper leaves it open: a coordinate with Q_jj = G_jj + mu = 0
    does not enter f at all (its column of B is zero and mu = 0); it is set
    to 0, one of its minimisers.
    """
    k = U.shape[1]
    Q = G + mu * np.eye(k)
    h = U @ Q - (R + mu * C)
    for j in range(k):
        if Q[j, j] > 0:
            new = np.maximum(U[:, j] - h[:, j] / Q[j, j], 0.0)
        else:
            new = np.zeros(U.shape[0])
        if upper is not None:
            new = np.minimum(new, upper)
        delta = new - U[:, j]
        U[:, j] = new
        h += np.outer(delta, Q[j, :])
    return U


def pgd_step_size(G, mu):
    """eta_t = 1 / (2 (L + mu_t)), L = max_j sum_l |G_lj| >= lambda_max(G).

    The paper requires only a diminishing step with sum eta = inf and
    sum eta^2 < inf (Theorem 1) and relates mu_t to 1/eta_t (Sec. 3.5.2);
    this choice keeps one step no longer than the inverse Lipschitz constant
    of the sketched gradient and decays like 1/(2 beta t).
    """
    L = np.max(np.sum(np.abs(G), axis=0))
    return 1.0 / (2.0 * (L + mu))


def pgd_step(U, G, R, eta, upper=None):
    """One projected-gradient step (eq. gradient_descent):
        U <- max(U - 2 eta [U B B^T - A B^T], 0)."""
    Unew = np.maximum(U - 2.0 * eta * (U @ G - R), 0.0)
    if upper is not None:
        Unew = np.minimum(Unew, upper)
    return Unew


def kkt_residual(U, C, G, R, mu):
    """Per-row relative projected-gradient norm of the regularised problem.

    Row i solves min_{u >= 0} 1/2 u Q u^T - q u^T with Q = G + mu I and
    q = r_i + mu c_i (eq. reg_sub divided by 2).  Its gradient is
    g = u Q - q; the projected gradient keeps g_j where u_j > 0 and min(g_j, 0)
    where u_j = 0.  The residual is ||pg|| / max(||q||, 1e-30); it is zero
    exactly at the row's unique minimiser when mu > 0.
    """
    k = G.shape[0]
    Q = G + mu * np.eye(k)
    q = R + mu * C
    g = U @ Q - q
    pg = np.where(U > 0, g, np.minimum(g, 0.0))
    return np.linalg.norm(pg, axis=1) / np.maximum(np.linalg.norm(q, axis=1), 1e-30)


def prox_cd_solve(U, C, G, R, mu, sweeps, tol=1e-4, max_sweeps=100, upper=None):
    """Run prox-CD sweeps on every row.

    sweeps >= 1: exactly that many sweeps (the paper uses one).
    sweeps == 0: sweep each row until its KKT residual is <= tol or
    max_sweeps sweeps are done.  Returns (U, sweeps_used_per_row).
    """
    U = np.array(U, dtype=np.float64, copy=True)
    rows = U.shape[0]
    if sweeps > 0:
        for _ in range(sweeps):
            prox_cd_sweep(U, C, G, R, mu, upper)
        return U, np.full(rows, sweeps, dtype=np.int64)
    used = np.zeros(rows, dtype=np.int64)
    active = kkt_residual(U, C, G, R, mu) > tol
    for _ in range(max_sweeps):
        if not active.any():
            break
        idx = np.nonzero(active)[0]
        Ua = U[idx]
        prox_cd_sweep(Ua, C[idx], G, R[idx], mu, upper)
        U[idx] = Ua
        used[idx] += 1
        active[idx] = kkt_residual(Ua, C[idx], G, R[idx], mu) > tol
    return U, used


def solve_subproblem(U, G, R, mu, cfg, upper=None):
    """The U (or V) update from the current factor and the sketched G, R."""
    C = np.array(U, dtype=np.float64, copy=True)
    if cfg.solver == SOLVER_PROX_CD:
        Unew, _ = prox_cd_solve(U, C, G, R, mu, cfg.sweeps, cfg.tol, cfg.max_sweeps, upper)
        return Unew
    if cfg.solver == SOLVER_PGD:
        return pgd_step(U, G, R, pgd_step_size(G, mu), upper)
    raise ValueError(cfg.solver)


# ----------------------------------------------------------------------------
# Half-iterations and the outer loop (Alg. 2, N = 1)
# ----------------------------------------------------------------------------

def box_upper(M, cfg):
    """Optional upper bound sqrt(2 ||M||_F) of eq. extra_con."""
    if not cfg.clip_upper:
        return None
    return math.sqrt(2.0 * frobenius(M))


def half_iteration(Mx, X, W, t, side, d, cfg, upper=None, rows=None):
    """Update X (rows of Mx) with W fixed: the U-step (side 0) or V-step (side 1).

    rows, if given, restricts the update to those rows of X; the subproblem
    is row-independent (eq. u_block), so the result on those rows is the same
    as with all rows present.
    """
    n_long = Mx.shape[1]
    S = sketch_matrix(cfg.sketch, cfg.seed, t, side, n_long, d)
    Msub = Mx if rows is None else Mx[rows]
    Xsub = X if rows is None else X[rows]
    if cfg.precision == "bf16" and not sp.issparse(S):
        # precision form: the sketch and M enter the products as bfloat16
        # values; the products themselves are exact here (FP64)
        S = _bf16.round_to_bf16(S)
        A = _bf16.round_to_bf16(Msub) @ S
        B = W.T @ S
    else:
        A, B = sketch_products(Msub, W, S)
    G, R = gram_and_rhs(A, B)
    return solve_subproblem(Xsub, G, R, mu_t(cfg, t), cfg, upper)


def update_U(M, U, V, t, cfg, upper=None, rows=None):
    """U^{t+1} from M, U^t, V^t (Alg. 2, U-side)."""
    return half_iteration(M, U, V, t, 0, cfg.d, cfg, upper, rows)


def update_V(M, U, V, t, cfg, upper=None, rows=None, Mt=None):
    """V^{t+1} from M^T, V^t and the current U (= U^{t+1}, Alg. 1).

    Mt, if given, is M^T already formed (a caller's cache; same values)."""
    if Mt is None:
        Mt = M.T.tocsr() if sp.issparse(M) else M.T
    return half_iteration(Mt, V, U, t, 1, cfg.d_prime, cfg, upper, rows)


def frobenius(M):
    """||M||_F."""
    if sp.issparse(M):
        return math.sqrt(math.fsum((M.data.astype(np.float64) ** 2).tolist()))
    return float(np.linalg.norm(np.asarray(M, dtype=np.float64)))


def relative_error(M, U, V):
    """||M - U V^T||_F / ||M||_F (Sec. 5.2).

    Dense M: the residual is formed entry by entry.  Sparse M: the residual
    norm is expanded as ||M||^2 - 2 sum_nnz M_ij <u_i, v_j> + <U^T U, V^T V>
    and each sum is taken with math.fsum.
    """
    normM = frobenius(M)
    if not sp.issparse(M):
        return float(np.linalg.norm(np.asarray(M) - U @ V.T)) / normM
    Mc = M.tocoo()
    cross = np.einsum("ij,ij->i", U[Mc.row], V[Mc.col])
    t1 = math.fsum((Mc.data.astype(np.float64) ** 2).tolist())
    t2 = math.fsum((Mc.data * cross).tolist())
    t3 = math.fsum(((U.T @ U) * (V.T @ V)).ravel().tolist())
    return math.sqrt(max(t1 - 2.0 * t2 + t3, 0.0)) / normM


def run(M, U0, V0, cfg, T, record=True):
    """T outer iterations of Alg. 2 with N = 1.

    Returns (U, V, errs) where errs[t] is the relative error after
    iteration t (U then V updated).
    """
    M = M.astype(np.float64) if not sp.issparse(M) else M.astype(np.float64).tocsr()
    U = np.array(U0, dtype=np.float64, copy=True)
    V = np.array(V0, dtype=np.float64, copy=True)
    upper = box_upper(M, cfg)
    errs = []
    for t in range(T):
        U = update_U(M, U, V, t, cfg, upper)
        V = update_V(M, U, V, t, cfg, upper)
        if record:
            errs.append(relative_error(M, U, V))
    return U, V, np.array(errs)
