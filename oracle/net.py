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


def loss_grad_scalar_perturbed(lam0, target_vals, w, b, c, layer=None, delta=0.0):
    """loss_grad_scalar with delta added to every eigenvalue image right after layer `layer`
    (x_{layer+1} += delta), the rest of the chain recomputed from there: the effect of one
    layer's output error on the loss and gradient."""
    xs = [np.asarray(lam0, dtype=np.float64)]
    for k in range(len(w)):
        x = xs[-1]
        y = w[k] * x * x + b[k] * x + c[k]
        if layer == k:
            y = y + delta
        xs.append(y)
    diff = xs[-1] - target_vals
    g = 2.0 * diff
    kk = len(w)
    dw, db, dc = np.zeros(kk), np.zeros(kk), np.zeros(kk)
    for k in range(kk - 1, -1, -1):
        x = xs[k]
        dw[k] = float(np.sum(g * x * x))
        db[k] = float(np.sum(g * x))
        dc[k] = float(np.sum(g))
        g = g * (2.0 * w[k] * x + b[k])
    return float(np.sum(diff * diff)), dw, db, dc, xs


def gradient_error_bound(lam0, target_vals, w, b, c, rel_err):
    """First-order bound of the error in (dL/dW, dL/dB, dL/dc) that layer outputs carrying
    errors of at most rel_err * max|x_{k+1}| (per eigenvalue) cause: for each layer the
    gradient is recomputed with every eigenvalue image shifted by +-that amount (the
    coherent, worst-sign case of the sums over eigenvalues), and the larger change is
    summed over the layers.  Returns three arrays (W, B, c)."""
    _, w0, b0, c0, xs = loss_grad_scalar_perturbed(lam0, target_vals, w, b, c)
    g0 = np.concatenate([w0, b0, c0])
    tot = np.zeros_like(g0)
    for k in range(len(w)):
        e = rel_err * float(np.abs(xs[k + 1]).max())
        worst = np.zeros_like(g0)
        for s in (1.0, -1.0):
            _, wp, bp, cp, _ = loss_grad_scalar_perturbed(lam0, target_vals, w, b, c, k, s * e)
            worst = np.maximum(worst, np.abs(np.concatenate([wp, bp, cp]) - g0))
        tot += worst
    kk = len(w)
    return tot[:kk], tot[kk:2 * kk], tot[2 * kk:]


def adam_scalar(lam0, target_vals, w, b, c, lr, steps, beta1=0.9, beta2=0.999, eps=1e-8):
    """Adam (Kingma and Ba, with bias-corrected moments) on the eigenvalue-space loss of the
    network, in FP64: the fit of the per-layer coefficients, written out step by step.
    Returns (loss before each step, final W, B, c)."""
    kk = len(w)
    p = np.concatenate([np.asarray(w, np.float64), np.asarray(b, np.float64), np.asarray(c, np.float64)])
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    losses = []
    for t in range(1, steps + 1):
        loss, dw, db, dc, _ = loss_grad_scalar(lam0, target_vals, p[:kk], p[kk:2 * kk], p[2 * kk:])
        losses.append(loss)
        g = np.concatenate([dw, db, dc])
        m = beta1 * m + (1.0 - beta1) * g
        v = beta2 * v + (1.0 - beta2) * g * g
        mhat = m / (1.0 - beta1 ** t)
        vhat = v / (1.0 - beta2 ** t)
        p = p - lr * mhat / (np.sqrt(vhat) + eps)
    return np.array(losses), p[:kk], p[kk:2 * kk], p[2 * kk:]
