"""Deep-NN SP2 recursion (test infrastructure, CPU FP64 NumPy).

Follows the paper's Alg. 1 step by step, in its notation:

    S_0 = W_0 H + B_0 with W_0 = -1/(e_N - e_1), B_0 = e_N/(e_N - e_1)   (reversed rescale)
    N_S = Tr S_0
    loop n = 1, 2, ...
        X_n     = f(S_{n-1})                       activation: the matrix square
        N_X     = Tr X_n
        IdErr_n = N_S - N_X
        sigma_n = Sign(|2 N_S - N_X - N_occ| - |N_X - N_occ| - sigma_{n-1} eps)
        S_n     = sigma_n X_n + (1 - sigma_n) S_{n-1}
        N_S     = sigma_n N_X + (1 - sigma_n) N_S
        stop if IdErr_n <= 0, or n > 2 and sigma_{n-1} != sigma_{n-2}
                and IdErr_n > 4.5 IdErr_{n-2}^2
    D = f_final(S_{m-1})                             (Eq. Refinement)

Readings taken where the text is silent (each listed in the design notes):
  * sigma_0 = 0, so the eps term is absent at the first layer;
  * Sign(0) (an exact tie) returns -sigma_{n-1}, or +1 when sigma_{n-1} = 0;
  * the refinement continues the alternation: its first composed step has sign
    -sigma_{m-1} (this equals the paper's sigma_{n-2} whenever the exit came from
    the alternation test); with sigma_{m-1} = 0 it starts with +1.
  * sign convention: Alg. 1's, i.e. sigma = +1 selects X^2 and sigma = -1 selects
    2X - X^2 (Eq. 10 and the appendix use the opposite labelling; the stopping rule
    only depends on whether consecutive signs differ).

The mixed-precision activation (Alg. 2) is emulated exactly: the two planes are
rounded with NumPy's float16 (round to nearest even) or an explicit round-to-nearest-
even truncation to bfloat16, their products are exact in FP64 and accumulated in FP64.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np

#: stopping constant of Alg. 1; the appendix bounds the two-step ratio by
#: C = (71 + 17 sqrt 17)/32 ~ 4.41 < 4.5.
STOP_FACTOR = 4.5


# --------------------------------------------------------------------------------------
# spectral bounds (the "spectral bound estimates" input of Alg. 1)
# --------------------------------------------------------------------------------------
def gershgorin(h: np.ndarray):
    """Gershgorin interval [min_i(H_ii - r_i), max_i(H_ii + r_i)], r_i = sum_{j!=i}|H_ij|.

    Widened outward by a bound on the FP64 summation error so that it encloses the
    spectrum of H as stored.
    """
    h = np.asarray(h, dtype=np.float64)
    n = h.shape[0]
    d = np.diag(h).copy()
    r = np.abs(h).sum(axis=1) - np.abs(d)
    slack = (2 * n + 4) * np.finfo(np.float64).eps
    r = r * (1.0 + slack) + slack * np.abs(d)
    lo = float(np.min(d - r))
    hi = float(np.max(d + r))
    return lo, hi


def rescale(h: np.ndarray, e1: float, en: float) -> np.ndarray:
    """Input layer S_0 = W_0 H + B_0 of Alg. 1: eigenvalues mapped to [0,1] in reverse order."""
    h = np.asarray(h, dtype=np.float64)
    w0 = -1.0 / (en - e1)
    b0 = en / (en - e1)
    return w0 * h + b0 * np.eye(h.shape[0])


# --------------------------------------------------------------------------------------
# activation functions
# --------------------------------------------------------------------------------------
def square_fp64(x: np.ndarray) -> np.ndarray:
    """f(X) = X^2 in FP64."""
    return x @ x


def round_bf16(x: np.ndarray) -> np.ndarray:
    """Round FP32 values to the nearest bfloat16 (ties to even), returned as float32.

    bfloat16 keeps the upper 16 bits of the FP32 encoding; rounding adds half of the
    dropped range plus the parity of the kept part before truncating.  Finite inputs only.
    """
    x32 = np.asarray(x, dtype=np.float32)
    u = x32.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def round_half(x: np.ndarray, fmt: str) -> np.ndarray:
    """FP16[.] or BF16[.] of FP32 values, returned as float32."""
    x32 = np.asarray(x, dtype=np.float32)
    if fmt == "fp16":
        return x32.astype(np.float16).astype(np.float32)
    if fmt == "bf16":
        return round_bf16(x32)
    raise ValueError(fmt)


def split_planes(x: np.ndarray, fmt: str = "fp16", scale_log2: int = 0):
    """Dual half-precision representation (Eqs. Split1, Split2) of the FP32 matrix X.

    X^(0) = FP16[X], X^(1) = FP16[X - X^(0)].  With scale_log2 = s > 0 both planes
    represent 2^s X (an exact power-of-two shift that keeps the low plane out of the
    half-precision subnormal range); s = 0 is the paper's split.  Returns the two
    planes as float32 arrays holding half-precision values, in units of 2^s.
    """
    xs = np.asarray(x, dtype=np.float32) * np.float32(2.0 ** scale_log2)
    x0 = round_half(xs, fmt)
    x1 = round_half(xs - x0, fmt)       # the difference is exact in FP32
    return x0, x1


def mixed_square(x: np.ndarray, fmt: str = "fp16", scale_log2: int = 0) -> np.ndarray:
    """Alg. 2 / Eq. Square: X^2 ~ X0 X0 + X0 X1 + (X0 X1)^T with the X1 X1 term dropped.

    For symmetric X the planes are symmetric and (X0 X1)^T = X1 X0.  Products of two
    half-precision numbers are exact in FP64; the sums are accumulated in FP64 (this is
    the exact-arithmetic reference the FP32-accumulating GPU kernel is compared to).
    The cross term is added as B + B^T so the result is exactly symmetric.
    """
    x0, x1 = split_planes(x, fmt, scale_log2)
    a = x0.astype(np.float64) @ x0.astype(np.float64)
    b = x0.astype(np.float64) @ x1.astype(np.float64)
    return (a + (b + b.T)) * (2.0 ** (-2 * scale_log2))


def mixed_square_rows(x: np.ndarray, rows, fmt: str = "fp16", scale_log2: int = 0) -> np.ndarray:
    """Selected rows of mixed_square (same definition, evaluated row by row for large X)."""
    x0, x1 = split_planes(x, fmt, scale_log2)
    x0 = x0.astype(np.float64)
    x1 = x1.astype(np.float64)
    r = np.asarray(rows)
    a = x0[r] @ x0
    b = x0[r] @ x1          # rows of X0 X1
    bt = x1[r] @ x0         # rows of X1 X0 = (X0 X1)^T for symmetric X
    return (a + (b + bt)) * (2.0 ** (-2 * scale_log2))


def mixed_square_fp32(fmt: str = "fp16", scale_log2: int = 0) -> Callable:
    """Activation returning FP32[mixed_square(X)] (the single-precision layer state)."""
    def f(x):
        return mixed_square(x, fmt, scale_log2).astype(np.float32).astype(np.float64)
    return f


# --------------------------------------------------------------------------------------
# Alg. 1
# --------------------------------------------------------------------------------------
def sign_with_tie(v: float, sigma_prev: int) -> int:
    """Sign of Alg. 1 with the tie reading: 0 -> -sigma_{n-1}, or +1 if sigma_{n-1} = 0."""
    if v > 0:
        return 1
    if v < 0:
        return -1
    return -sigma_prev if sigma_prev != 0 else 1


def refinement(s: np.ndarray, first_sign: int) -> np.ndarray:
    """Eq. Refinement: two composed SP2 layers in FP64.

    first_sign = +1: 2 S^2 - S^4 (square, then 2Y - Y^2);
    first_sign = -1: (2 S - S^2)^2 (2S - S^2, then square).
    """
    s = np.asarray(s, dtype=np.float64)
    s2 = s @ s
    if first_sign > 0:
        return 2.0 * s2 - s2 @ s2
    y = 2.0 * s - s2
    return y @ y


@dataclass
class SP2Result:
    d: np.ndarray                      # density matrix after refinement (FP64)
    layers: int                        # m, the exit layer of Alg. 1
    converged: bool
    sigma: list = field(default_factory=list)   # sigma_1..sigma_m
    iderr: list = field(default_factory=list)   # IdErr_1..IdErr_m
    ns: list = field(default_factory=list)      # N_S entering layer n (Tr S_{n-1})
    nx: list = field(default_factory=list)      # N_X of layer n (Tr X_n)
    s_last: Optional[np.ndarray] = None         # S_{m-1}
    bounds: tuple = (float("nan"), float("nan"))
    first_sign: int = 0


def sp2_alg1(h: np.ndarray, n_occ: int, eps: float = 0.0, bounds=None, max_layers: int = 100,
             activation: Callable = square_fp64, refine: bool = True) -> SP2Result:
    """Alg. 1 (Deep-NN SP2) on the matrix H; FP64 unless another activation is passed.

    Returns the refined density matrix f_final(S_{m-1}) and the per-layer history.
    If max_layers is reached without meeting a stopping test, S_{max_layers} is refined
    and `converged` is False.
    """
    h = np.asarray(h, dtype=np.float64)
    e1, en = bounds if bounds is not None else gershgorin(h)
    s_prev = rescale(h, e1, en)                      # S_0
    n_s = float(np.trace(s_prev))                    # N_S = Tr S_0
    res = SP2Result(d=None, layers=0, converged=False, bounds=(e1, en))
    sig = [0]                                         # sigma_0 = 0
    iderr = [float("nan")]                           # 1-based history
    n = 0
    while True:
        n += 1
        if n > max_layers:
            res.layers = n - 1
            break
        x = activation(s_prev)                       # X_n = f(S_{n-1})
        n_x = float(np.trace(x))                     # N_X = Tr X_n
        e_n = n_s - n_x                              # IdErr_n
        v = abs(2.0 * n_s - n_x - n_occ) - abs(n_x - n_occ) - sig[n - 1] * eps
        s_n_sign = sign_with_tie(v, sig[n - 1])
        res.ns.append(n_s)
        res.nx.append(n_x)
        res.iderr.append(e_n)
        res.sigma.append(s_n_sign)
        sig.append(s_n_sign)
        iderr.append(e_n)
        s_new = s_n_sign * x + (1 - s_n_sign) * s_prev          # W_n X_n + B_n
        n_s = s_n_sign * n_x + (1 - s_n_sign) * n_s
        stop = e_n <= 0.0 or (n > 2 and sig[n - 1] != sig[n - 2]
                               and e_n > STOP_FACTOR * iderr[n - 2] ** 2)
        if stop:
            res.layers = n
            res.converged = True
            break
        s_prev = s_new
    # s_prev is S_{m-1} on convergence, S_{max_layers} otherwise
    res.s_last = s_prev
    last = sig[res.layers - 1] if res.converged else sig[res.layers]
    res.first_sign = -last if last != 0 else 1
    res.d = refinement(s_prev, res.first_sign) if refine else s_prev.copy()
    return res


def sp2_eigen(lam0: np.ndarray, n_occ: int, eps: float = 0.0, max_layers: int = 100) -> SP2Result:
    """Alg. 1 applied to the eigenvalues of S_0 (every S_n is a polynomial in H, so
    its eigenvalues follow the scalar maps x^2 and 2x - x^2).  FP64, O(N m).

    `d` holds the refined eigenvalues f_final(lambda^{(m-1)}).
    """
    lam = np.asarray(lam0, dtype=np.float64).copy()
    n_s = float(np.sum(lam))
    res = SP2Result(d=None, layers=0, converged=False)
    sig = [0]
    iderr = [float("nan")]
    n = 0
    while True:
        n += 1
        if n > max_layers:
            res.layers = n - 1
            break
        x = lam * lam
        n_x = float(np.sum(x))
        e_n = n_s - n_x
        v = abs(2.0 * n_s - n_x - n_occ) - abs(n_x - n_occ) - sig[n - 1] * eps
        s_n_sign = sign_with_tie(v, sig[n - 1])
        res.ns.append(n_s)
        res.nx.append(n_x)
        res.iderr.append(e_n)
        res.sigma.append(s_n_sign)
        sig.append(s_n_sign)
        iderr.append(e_n)
        new = x if s_n_sign > 0 else 2.0 * lam - x
        n_s = s_n_sign * n_x + (1 - s_n_sign) * n_s
        stop = e_n <= 0.0 or (n > 2 and sig[n - 1] != sig[n - 2]
                               and e_n > STOP_FACTOR * iderr[n - 2] ** 2)
        if stop:
            res.layers = n
            res.converged = True
            break
        lam = new
    res.s_last = lam
    last = sig[res.layers - 1] if res.converged else sig[res.layers]
    res.first_sign = -last if last != 0 else 1
    if res.first_sign > 0:
        y = lam * lam
        res.d = 2.0 * y - y * y
    else:
        y = 2.0 * lam - lam * lam
        res.d = y * y
    return res


def theorem_constant() -> float:
    """C = (71 + 17 sqrt 17)/32 of the appendix theorem."""
    return (71.0 + 17.0 * math.sqrt(17.0)) / 32.0

