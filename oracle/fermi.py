"""Optimized finite-temperature SP2 expansion (Sec. "Optimized SP2 Finite Temperature
Fermi-Operator Expansion"), CPU FP64 NumPy.  Test infrastructure: imported only by tests
and the CPU leg of the benchmark.

Model (Eq. general SP2 and the read-out that follows it), for a rescaled energy
eps in [0, 1]:

    eps_0 = eps
    eps_n = theta_{n-1,1} eps_{n-1}^2 + theta_{n-1,2} eps_{n-1} + theta_{n-1,3},   n = 1..L
    F~(eps) = 1 - sum_{i=0}^{L} c_i eps_i

fitted to the Fermi function F(eps) = 1 / (exp(beta (eps - mu)) + 1) (Eq. fermi, mu = 1/2
there) by minimizing the weighted sum of squares  sum_i w_i [F~(eps_i) - F(eps_i)]^2  over a
grid on [0, 1] with Levenberg-Marquardt.

Readings where the section is silent (each listed in the design notes):
  * grid: m equally spaced points on [0, 1] with trapezoid weights, so the loss
    approximates the integral of the squared error;
  * start: the truncated SP2 expansion whose branch (x^2 or 2x - x^2) at each layer
    keeps the image of mu closest to 1/2 (x^2 on a tie), read out as F~ = 1 - eps_L;
  * Levenberg-Marquardt in Marquardt's form: solve (J^T J + lambda diag(J^T J)) d = -J^T r,
    accept a step that lowers the loss and divide lambda by 10, otherwise multiply it
    by 10; start at lambda = 1e-3, stop after max_iter steps or when lambda > 1e12.
  * on matrices, eps is the spectrum of X_0 = (H - e_1 I)/(e_N - e_1) (lowest energy at
    0, so F ~ 1 on the occupied side), and D = I - sum_i c_i X_i.
"""
from __future__ import annotations

import numpy as np


def fermi(eps, beta: float = 40.0, mu: float = 0.5):
    """Eq. fermi: F(eps) = 1 / (exp(beta (eps - mu)) + 1), evaluated without overflow."""
    x = beta * (np.asarray(eps, dtype=np.float64) - mu)
    out = np.empty_like(x)
    pos = x > 0
    ex = np.exp(-x[pos])
    out[pos] = ex / (1.0 + ex)
    out[~pos] = 1.0 / (1.0 + np.exp(x[~pos]))
    return out


def layers_scalar(eps, theta):
    """eps_0 .. eps_L of Eq. general SP2 (theta has shape (L, 3)); returns (L + 1, m)."""
    e = [np.asarray(eps, dtype=np.float64)]
    for t1, t2, t3 in np.asarray(theta, dtype=np.float64):
        x = e[-1]
        e.append(t1 * x * x + t2 * x + t3)
    return np.array(e)


def model_scalar(eps, theta, c):
    """F~(eps) = 1 - sum_i c_i eps_i."""
    e = layers_scalar(eps, theta)
    return 1.0 - np.asarray(c, dtype=np.float64) @ e


def model_matrix(h, theta, c, e1: float, en: float):
    """The same network on a symmetric matrix: X_0 = (H - e1 I)/(en - e1),
    X_{k+1} = theta_{k,1} X_k^2 + theta_{k,2} X_k + theta_{k,3} I, D = I - sum_i c_i X_i."""
    h = np.asarray(h, dtype=np.float64)
    n = h.shape[0]
    eye = np.eye(n)
    x = (h - e1 * eye) / (en - e1)
    c = np.asarray(c, dtype=np.float64)
    d = eye - c[0] * x
    for k, (t1, t2, t3) in enumerate(np.asarray(theta, dtype=np.float64)):
        x = t1 * (x @ x) + t2 * x + t3 * eye
        d = d - c[k + 1] * x
    return d


def grid(m: int):
    """m equally spaced points on [0, 1] and their trapezoid weights (sum 1)."""
    x = np.linspace(0.0, 1.0, m)
    w = np.full(m, 1.0 / (m - 1))
    w[0] = w[-1] = 0.5 / (m - 1)
    return x, w


def pack(theta, c):
    return np.concatenate([np.asarray(theta, dtype=np.float64).ravel(), np.asarray(c, dtype=np.float64)])


def unpack(p, layers: int):
    p = np.asarray(p, dtype=np.float64)
    return p[:3 * layers].reshape(layers, 3), p[3 * layers:]


def residuals(p, layers: int, x, w, target):
    theta, c = unpack(p, layers)
    return np.sqrt(w) * (model_scalar(x, theta, c) - target)


def loss(p, layers: int, x, w, target) -> float:
    """Weighted sum of squares; inf or nan for a trial step that overflows (then rejected)."""
    with np.errstate(over="ignore", invalid="ignore"):
        r = residuals(p, layers, x, w, target)
        return float(r @ r)


def jacobian(p, layers: int, x, w):
    """d residual / d parameter by the chain rule backwards through the layers:
    dF~/dc_i = -eps_i; with g_L = -c_L and g_k = -c_k + g_{k+1} (2 theta_{k,1} eps_k + theta_{k,2}),
    dF~/dtheta_{k,.} = g_{k+1} (eps_k^2, eps_k, 1)."""
    theta, c = unpack(p, layers)
    e = layers_scalar(x, theta)                 # (L + 1, m)
    m = x.shape[0]
    jac = np.zeros((m, 4 * layers + 1))
    jac[:, 3 * layers:] = -e.T
    g = -c[layers] * np.ones(m)
    for k in range(layers - 1, -1, -1):
        ek = e[k]
        jac[:, 3 * k + 0] = g * ek * ek
        jac[:, 3 * k + 1] = g * ek
        jac[:, 3 * k + 2] = g
        g = -c[k] + g * (2.0 * theta[k, 0] * ek + theta[k, 1])
    return np.sqrt(w)[:, None] * jac


def truncated_sp2_start(layers: int, mu: float = 0.5):
    """Truncated SP2 start: at each layer the branch that keeps the image of mu closest to
    1/2 (x^2 on a tie); read-out F~ = 1 - eps_L."""
    theta = np.zeros((layers, 3))
    m = mu
    for k in range(layers):
        sq, pr = m * m, 2.0 * m - m * m
        if abs(sq - 0.5) <= abs(pr - 0.5):
            theta[k] = (1.0, 0.0, 0.0)
            m = sq
        else:
            theta[k] = (-1.0, 2.0, 0.0)
            m = pr
    c = np.zeros(layers + 1)
    c[layers] = 1.0
    return theta, c


def lm_fit(layers: int, beta: float = 40.0, mu: float = 0.5, m: int = 1001, max_iter: int = 300,
           theta0=None, c0=None):
    """Levenberg-Marquardt fit of (theta, c) to the Fermi function on the grid.
    Returns (theta, c, final loss, iterations run, loss history)."""
    x, w = grid(m)
    target = fermi(x, beta, mu)
    if theta0 is None:
        theta0, c0 = truncated_sp2_start(layers, mu)
    p = pack(theta0, c0)
    cur = loss(p, layers, x, w, target)
    hist = [cur]
    lam = 1e-3
    it = 0
    while it < max_iter and lam <= 1e12:
        it += 1
        r = residuals(p, layers, x, w, target)
        jac = jacobian(p, layers, x, w)
        a = jac.T @ jac
        g = jac.T @ r
        step = np.linalg.solve(a + lam * np.diag(np.diag(a)), -g)
        trial = p + step
        new = loss(trial, layers, x, w, target)
        if new < cur:
            p, cur = trial, new
            lam /= 10.0
        else:
            lam *= 10.0
        hist.append(cur)
    theta, c = unpack(p, layers)
    return theta, c, cur, it, hist
