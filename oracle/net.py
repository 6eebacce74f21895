"""Generalized SP2 network (test infrastructure, CPU FP64 NumPy).

Eq. general SP2 replaces the two SP2 polynomials x^2 and 2x - x^2 by a general
second-degree polynomial per layer.  Applied to a matrix this is the layer

    X_{k+1} = W_k X_k^2 + B_k X_k + c_k I,        k = 0 .. K-1

with trainable scalars (W_k, B_k, c_k) = (theta_{k,1}, theta_{k,2}, theta_{k,3}).
The loss is the squared Frobenius distance of X_K to a target T; with T a function
of the same Hamiltonian (the Fermi-Dirac matrix of Eq. 1) and X_0 an affine map of
H, every X_k shares T's eigenbasis and the loss equals the sum over eigenvalues of
the scalar recursion's squared error -- a weighted grid loss in the sense of the
paper's training objective, with the eigenvalues as the grid.

The gradient below is derived by hand (reverse-mode chain rule):
    G_K      = 2 (X_K - T)
    dL/dW_k  = <G_{k+1}, X_k^2>_F
    dL/dB_k  = <G_{k+1}, X_k>_F
    dL/dc_k  = Tr G_{k+1}
    G_k      = W_k (G_{k+1} X_k + X_k G_{k+1}) + B_k G_{k+1}
"""
from __future__ import annotations

import numpy as np


def sp2_branch_coefficients(sigmas):
    """(W, B, c) reproducing SP2 layers: sigma=+1 -> x^2 = (1,0,0); sigma=-1 -> 2x - x^2 = (-1,2,0)."""
    w = np.array([1.0 if s > 0 else -1.0 for s in sigmas])
    b = np.array([0.0 if s > 0 else 2.0 for s in sigmas])
    c = np.zeros(len(sigmas))
    return w, b, c


def forward_matrix(x0, w, b, c):
    """All layers X_0 .. X_K of the matrix network in FP64."""
    xs = [np.asarray(x0, dtype=np.float64)]
    eye = np.eye(xs[0].shape[0])
    for k in range(len(w)):
        x = xs[-1]
        xs.append(w[k] * (x @ x) + b[k] * x + c[k] * eye)
    return xs


def forward_scalar(lam0, w, b, c):
    """The same recursion on eigenvalues: x_{k+1} = W_k x_k^2 + B_k x_k + c_k."""
    xs = [np.asarray(lam0, dtype=np.float64)]
    for k in range(len(w)):
        x = xs[-1]
        xs.append(w[k] * x * x + b[k] * x + c[k])
    return xs


def loss_grad_matrix(x0, target, w, b, c):
    """Loss ||X_K - T||_F^2 and its gradient w.r.t. (W, B, c) and X_0, by the matrix adjoint."""
    xs = forward_matrix(x0, w, b, c)
    kk = len(w)
    diff = xs[-1] - target
    loss = float(np.sum(diff * diff))
    g = 2.0 * diff
    dw = np.zeros(kk)
    db = np.zeros(kk)
    dc = np.zeros(kk)
    for k in range(kk - 1, -1, -1):
        x = xs[k]
        dw[k] = float(np.sum(g * (x @ x)))
        db[k] = float(np.sum(g * x))
        dc[k] = float(np.trace(g))
        g = w[k] * (g @ x + x @ g) + b[k] * g
    return loss, dw, db, dc, g


def loss_grad_scalar(lam0, target_vals, w, b, c):
    """Loss sum_j (x_K(lam_j) - t_j)^2 and its gradient, on eigenvalues."""
    xs = forward_scalar(lam0, w, b, c)
    kk = len(w)
    diff = xs[-1] - target_vals
    loss = float(np.sum(diff * diff))
    g = 2.0 * diff
    dw = np.zeros(kk)
    db = np.zeros(kk)
    dc = np.zeros(kk)
    for k in range(kk - 1, -1, -1):
        x = xs[k]
        dw[k] = float(np.sum(g * x * x))
        db[k] = float(np.sum(g * x))
        dc[k] = float(np.sum(g))
        g = g * (2.0 * w[k] * x + b[k])
    return loss, dw, db, dc, g


def loss_scalar(lam0, target_vals, w, b, c):
    xs = forward_scalar(lam0, w, b, c)
    d = xs[-1] - target_vals
    return float(np.sum(d * d))


def finite_difference_grad(lam0, target_vals, w, b, c, h=1e-4):
    """Central differences of loss_scalar w.r.t. every coefficient (step h, FP64)."""
    out = []
    for arr_idx in range(3):
        params = [np.array(w, dtype=np.float64), np.array(b, dtype=np.float64),
                  np.array(c, dtype=np.float64)]
        g = np.zeros(len(w))
        for k in range(len(w)):
            pp = [p.copy() for p in params]
            pm = [p.copy() for p in params]
            pp[arr_idx][k] += h
            pm[arr_idx][k] -= h
            g[k] = (loss_scalar(lam0, target_vals, *pp) - loss_scalar(lam0, target_vals, *pm)) / (2 * h)
        out.append(g)
    return out
