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
# spectral bounds (the estimated spectral range that Alg. 1 takes as input)
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



# --------------------------------------------------------------------------------------
# Accelerated Deep-NN SP2 (Sec. "Accelerated Deep-NN SP2")
# --------------------------------------------------------------------------------------
#: accelerated layers are used while the tracked bounds leave a distance larger than
#: this to the fixed points (max(l, 1 - h) > ACCEL_SWITCH); Alg. 1 continues from there
ACCEL_SWITCH = 0.01


def quadratic_range(a: float, b: float, c: float, lo: float, hi: float):
    """(min, max) of a x^2 + b x + c over [lo, hi]: the endpoints and, if inside, the vertex."""
    pts = [lo, hi]
    if a != 0.0:
        x = -b / (2.0 * a)
        if lo < x < hi:
            pts.append(x)
    vals = [a * x * x + b * x + c for x in pts]
    return min(vals), max(vals)


def accelerated_layer(l: float, h: float):
    """One accelerated layer: the continuous weight sigma_n and the rescale that follows.

    Reading of the section (its coefficients are given only in a script that is not
    part of the paper): with the unoccupied eigenvalues of S_{n-1} in [0, l] and the
    occupied ones in [h, 1] (l < h; S_0 reverses the order of H), the layer applies the
    projection p(x) = sigma x^2 + (1 - sigma) x, i.e. W = sigma I and B = (1 - sigma) S_{n-1}
    on X_n = S_{n-1}^2 as in Alg. 1 but with sigma real, then shifts and rescales the
    range of p over [0, 1] back onto [0, 1].  sigma is chosen to separate the images of
    the two intervals as far as possible (min over [h, 1] minus max over [0, l]) without
    letting them cross.

    For sigma >= 1 the rescaled map is ((x - v)/(1 - v))^2 with vertex v = (sigma - 1)/(2 sigma);
    the separation [(h - v)^2 - max(v, l - v)^2]/(1 - v)^2 increases in v up to
    h + l - 1 and decreases for v > l/2, so v = clamp(h + l - 1, 0, l/2).  For sigma <= -1
    the map is the mirror image x -> 1 - q(1 - x) with the roles of l and 1 - h
    exchanged.  The branch with the larger separation is taken (the x^2 side on a tie).

    Returns (sigma, W, B_s, B_i, l_new, h_new): S_n = W X_n + B_s S_{n-1} + B_i I.
    """
    best = None
    for branch in (1, -1):
        if branch > 0:
            v = min(max(h + l - 1.0, 0.0), l / 2.0)
        else:
            v = min(max(1.0 - h - l, 0.0), (1.0 - h) / 2.0)
        sigma = branch / (1.0 - 2.0 * v)
        # rescale: the range of p over [0, 1] is mapped onto [0, 1]
        pmin, pmax = quadratic_range(sigma, 1.0 - sigma, 0.0, 0.0, 1.0)
        w = sigma / (pmax - pmin)
        bs = (1.0 - sigma) / (pmax - pmin)
        bi = -pmin / (pmax - pmin)
        # images of the bounding intervals under the rescaled layer
        _, l_new = quadratic_range(w, bs, bi, 0.0, l)
        h_new, _ = quadratic_range(w, bs, bi, h, 1.0)
        cand = (sigma, w, bs, bi, l_new, h_new)
        if best is None or (h_new - l_new) > (best[5] - best[4]):
            best = cand
    return best


def homo_lumo_rescaled(homo: float, lumo: float, e1: float, en: float):
    """Bounds of the rescaled spectrum of S_0: unoccupied in [0, l0], occupied in [h0, 1]."""
    return (en - lumo) / (en - e1), (en - homo) / (en - e1)


@dataclass
class SP2AccResult(SP2Result):
    accelerated: int = 0                             # layers 1..accelerated used sigma_n in R
    gap_violation: int = 0                           # first layer whose consistency check failed
    sigma_c: list = field(default_factory=list)     # continuous sigma_n of layer n
    lh: list = field(default_factory=list)           # (l, h) entering layer n


def sp2_accelerated(h: np.ndarray, n_occ: int, homo: float, lumo: float, bounds=None, eps: float = 0.0,
                    max_layers: int = 100, activation: Callable = square_fp64, refine: bool = True,
                    switch: float = ACCEL_SWITCH, noise_rel: float = 1e-8) -> SP2AccResult:
    """Accelerated Deep-NN SP2 on the matrix H.

    Every occupied eigenvalue of H is <= homo and every unoccupied one >= lumo (an
    interval inside the HOMO-LUMO gap, the prior knowledge the section requires).
    Layers use `accelerated_layer` while max(l, 1 - h) > switch, then Alg. 1's own
    sign rule; the parameter-free stopping test of Alg. 1 is applied as printed, except
    that its second clause compares IdErr_n with IdErr_{n-2} only when the two layers
    between them were ordinary SP2 layers (the bound behind it holds for x^2 and
    2x - x^2).  The refinement is Eq. Refinement, as for Alg. 1.

    Consistency of the interval: if it lies inside the gap, exactly N_occ eigenvalues of S_0
    are in [h, 1] and the rest in [0, l]; every layer (accelerated or not) maps those
    intervals onto the tracked ones, so |Tr S_{n-1} - N_occ| <= (N - N_occ) l + N_occ (1 - h)
    at every layer.  The first layer where this fails by more than noise_rel N is recorded
    in `gap_violation` (the interval was not inside the gap).
    """
    h = np.asarray(h, dtype=np.float64)
    e1, en = bounds if bounds is not None else gershgorin(h)
    l, hh = homo_lumo_rescaled(homo, lumo, e1, en)
    accel = 0.0 <= l < hh <= 1.0
    s_prev = rescale(h, e1, en)                      # S_0
    res = SP2AccResult(d=None, layers=0, converged=False, bounds=(e1, en))
    sig = [0]
    iderr = [float("nan")]
    last_acc = 0
    n = 0
    while True:
        n += 1
        if n > max_layers:
            res.layers = n - 1
            break
        n_s = float(np.trace(s_prev))                # Tr S_{n-1}
        x = activation(s_prev)                       # X_n = f(S_{n-1})
        n_x = float(np.trace(x))
        e_n = n_s - n_x
        res.ns.append(n_s)
        res.nx.append(n_x)
        res.iderr.append(e_n)
        res.lh.append((l, hh))
        nn = h.shape[0]
        if accel and not res.gap_violation and \
                abs(n_s - n_occ) > (nn - n_occ) * l + n_occ * (1.0 - hh) + noise_rel * nn:
            res.gap_violation = n
        if accel and max(l, 1.0 - hh) > switch:
            sigma, w, bs, bi, l, hh = accelerated_layer(l, hh)
            s_sign = 1 if sigma > 0 else -1
            last_acc = n
            s_new = w * x + bs * s_prev + bi * np.eye(h.shape[0])
        else:
            v = abs(2.0 * n_s - n_x - n_occ) - abs(n_x - n_occ) - sig[n - 1] * eps
            s_sign = sign_with_tie(v, sig[n - 1])
            sigma = float(s_sign)
            s_new = s_sign * x + (1 - s_sign) * s_prev
            if accel:   # the tracked intervals follow the SP2 maps too
                l, hh = (l * l, hh * hh) if s_sign > 0 else (2.0 * l - l * l, 2.0 * hh - hh * hh)
        res.sigma.append(s_sign)
        res.sigma_c.append(sigma)
        sig.append(s_sign)
        iderr.append(e_n)
        stop = e_n <= 0.0 or (n > 2 and n >= last_acc + 3 and sig[n - 1] != sig[n - 2]
                               and e_n > STOP_FACTOR * iderr[n - 2] ** 2)
        if stop:
            res.layers = n
            res.converged = True
            break
        s_prev = s_new
    res.accelerated = min(last_acc, res.layers)
    res.s_last = s_prev
    last = sig[res.layers - 1] if res.converged else sig[res.layers]
    res.first_sign = -last if last != 0 else 1
    res.d = refinement(s_prev, res.first_sign) if refine else s_prev.copy()
    return res


def sp2_eigen_accelerated(lam0: np.ndarray, n_occ: int, l0: float, h0: float, eps: float = 0.0,
                          max_layers: int = 100, switch: float = ACCEL_SWITCH,
                          noise_rel: float = 1e-8) -> SP2AccResult:
    """`sp2_accelerated` on the eigenvalues of S_0 (each layer is a quadratic in S_{n-1},
    so the eigenvalues follow the scalar maps).  FP64, O(N m).  `d` holds the refined
    eigenvalues."""
    lam = np.asarray(lam0, dtype=np.float64).copy()
    l, hh = l0, h0
    accel = 0.0 <= l < hh <= 1.0
    res = SP2AccResult(d=None, layers=0, converged=False)
    sig = [0]
    iderr = [float("nan")]
    last_acc = 0
    n = 0
    while True:
        n += 1
        if n > max_layers:
            res.layers = n - 1
            break
        n_s = float(np.sum(lam))
        x = lam * lam
        n_x = float(np.sum(x))
        e_n = n_s - n_x
        res.ns.append(n_s)
        res.nx.append(n_x)
        res.iderr.append(e_n)
        res.lh.append((l, hh))
        nn = lam.size
        if accel and not res.gap_violation and \
                abs(n_s - n_occ) > (nn - n_occ) * l + n_occ * (1.0 - hh) + noise_rel * nn:
            res.gap_violation = n
        if accel and max(l, 1.0 - hh) > switch:
            sigma, w, bs, bi, l, hh = accelerated_layer(l, hh)
            s_sign = 1 if sigma > 0 else -1
            last_acc = n
            new = w * x + bs * lam + bi
        else:
            v = abs(2.0 * n_s - n_x - n_occ) - abs(n_x - n_occ) - sig[n - 1] * eps
            s_sign = sign_with_tie(v, sig[n - 1])
            sigma = float(s_sign)
            new = x if s_sign > 0 else 2.0 * lam - x
            if accel:
                l, hh = (l * l, hh * hh) if s_sign > 0 else (2.0 * l - l * l, 2.0 * hh - hh * hh)
        res.sigma.append(s_sign)
        res.sigma_c.append(sigma)
        sig.append(s_sign)
        iderr.append(e_n)
        stop = e_n <= 0.0 or (n > 2 and n >= last_acc + 3 and sig[n - 1] != sig[n - 2]
                               and e_n > STOP_FACTOR * iderr[n - 2] ** 2)
        if stop:
            res.layers = n
            res.converged = True
            break
        lam = new
    res.accelerated = min(last_acc, res.layers)
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


# --------------------------------------------------------------------------------------
# HOMO/LUMO estimates from a finished expansion (for the accelerated layers of a later
# call, Sec. Accelerated Deep-NN SP2: the estimates can come from previous expansions)
# --------------------------------------------------------------------------------------
def estimate_gap(sigma_c, iderr, layers: int, emin: float, emax: float, n: int, floor_rel: float,
                 upper: float = 0.25, margin: float = 0.1):
    """(homo, lumo) estimated from the history of a converged run, or None.

    Reading (the section refers to this possibility without a method): near convergence
    IdErr_k = Tr[S_{k-1} - S_{k-1}^2] is dominated by the two eigenvalues nearest the step,
    the LUMO image a (near 0) and the HOMO image 1 - c (near 1): IdErr_k ~ a + c.  An
    ordinary layer maps (a, c) to (a^2, 2c - c^2) (x^2) or (2a - a^2, c^2) (2x - x^2), so two
    consecutive values give a quadratic for a (x^2: a^2 - 2a + (2 IdErr_k - IdErr_{k+1}) = 0)
    and c = IdErr_k - a (the 2x - x^2 case with the roles exchanged).  The layer maps before
    S_{k-1} (sigma_n, with the shift v = (1 - 1/|sigma_n|)/2 of an accelerated layer) are
    inverted exactly on their increasing branch, and S_0 = (emax I - H)/(emax - emin) gives the
    energies.  Other eigenvalues near the step add to IdErr and move both estimates toward
    the middle of the gap.  Every consecutive pair with IdErr_k <= upper, IdErr_{k+1} >=
    floor_rel n and an ordinary layer k contributes; the highest HOMO and the lowest LUMO
    estimate are kept, then each is moved inward by `margin` times their distance.
    """
    maps = []
    for s in list(sigma_c)[:max(layers - 1, 0)]:
        b = 1 if s > 0 else -1
        maps.append((b, 0.5 * (1.0 - 1.0 / abs(s))))

    def inverse(y, b, v):
        y = min(max(y, 0.0), 1.0)
        if b > 0:                                   # y = ((x - v)/(1 - v))^2, x >= v
            return v + (1.0 - v) * math.sqrt(y)
        return (1.0 - v) * (1.0 - math.sqrt(1.0 - y))   # y = 1 - ((1 - v - x)/(1 - v))^2

    homos, lumos = [], []
    span = emax - emin
    for k in range(len(maps) - 1):
        e0, e1 = iderr[k], iderr[k + 1]
        b, v = maps[k]
        if not (e0 <= upper and e1 >= floor_rel * n and v == 0.0):
            continue
        disc = 1.0 - (2.0 * e0 - e1)
        if disc < 0.0:
            continue
        r = 1.0 - math.sqrt(disc)
        a, c = (r, e0 - r) if b > 0 else (e0 - r, r)
        if a <= 0.0 or c <= 0.0:
            continue
        xl, xh = a, 1.0 - c
        for bb, vv in reversed(maps[:k]):
            xl, xh = inverse(xl, bb, vv), inverse(xh, bb, vv)
        homos.append(emax - xh * span)
        lumos.append(emax - xl * span)
    if not homos:
        return None
    homo, lumo = max(homos), min(lumos)
    if lumo <= homo:
        return None
    w = lumo - homo
    return homo + margin * w, lumo - margin * w
