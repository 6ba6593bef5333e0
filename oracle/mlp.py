"""FP64 reference of the warm-start network (test infrastructure).

A learned warm start for the to-tolerance NNLS solves of the sketched
subproblem: a two-layer perceptron maps the sketched row a_i (d values,
sparse for a subsampling sketch) and the current row u_i^t (k values) to a
starting point for prox-CD,
    h = ReLU(a_i W1a + W1u u_i + b1)        (hidden width H)
    y = ReLU(W2 h + b2)                     (k outputs, nonnegative)
With residual=True a variant adds u_i^t to the output pre-activation,
    y = ReLU(u_i + W2 h + b2),
so that the second layer predicts a correction to the cold start u_i^t.
It is trained with the mean squared error against the rows' NNLS solutions and
the Adam optimiser (Kingma and Ba, "Adam: a method for stochastic
optimization", ICLR 2015).  The paper has no such network; this module is
the plain definition the GPU kernels are checked against.

Shapes: W1a is d x H (row c = weights of input column c), W1u is H x k,
b1 is H, W2 is k x H, b2 is k.  A batch is (A, U, Y) with A a scipy CSR
matrix (rows x d), U and Y dense (rows x k).  The derivative of ReLU at 0
is taken as 0.
"""
import numpy as np

PARAMS = ("W1a", "W1u", "b1", "W2", "b2")


def forward(p, A, U, residual=False):
    """Returns (Hpre, H, Ypre, Y)."""
    Hpre = np.asarray(A @ p["W1a"]) + U @ p["W1u"].T + p["b1"]
    H = np.maximum(Hpre, 0.0)
    Ypre = H @ p["W2"].T + p["b2"]
    if residual:
        Ypre = Ypre + U
    return Hpre, H, Ypre, np.maximum(Ypre, 0.0)


def loss(Yhat, Y):
    """L = (1/B) sum_b ||yhat_b - y_b||^2."""
    return float(np.sum((Yhat - Y) ** 2) / Y.shape[0])


def backward(p, A, U, Y, residual=False):
    """Gradients of loss(forward(p, A, U, residual)[3], Y) with respect to
    every parameter (u_i^t is an input, so the residual path adds none)."""
    Hpre, H, Ypre, Yhat = forward(p, A, U, residual)
    B = Y.shape[0]
    dY = (2.0 / B) * (Yhat - Y) * (Ypre > 0)
    g = {"W2": dY.T @ H, "b2": dY.sum(axis=0)}
    dH = (dY @ p["W2"]) * (Hpre > 0)
    g["W1u"] = dH.T @ U
    g["W1a"] = np.asarray(A.T @ dH)
    g["b1"] = dH.sum(axis=0)
    return g, loss(Yhat, Y)


def adam_step(p, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (t counts from 1), in place on p, m and v."""
    for name in PARAMS:
        m[name] = beta1 * m[name] + (1.0 - beta1) * g[name]
        v[name] = beta2 * v[name] + (1.0 - beta2) * g[name] ** 2
        mhat = m[name] / (1.0 - beta1 ** t)
        vhat = v[name] / (1.0 - beta2 ** t)
        p[name] = p[name] - lr * mhat / (np.sqrt(vhat) + eps)
    return p, m, v
