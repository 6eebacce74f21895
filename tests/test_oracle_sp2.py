"""Pins of the SP2 oracle (Alg. 1, Alg. 2, Eq. Refinement, appendix theorem) against
the exact density matrix, closed forms, brute force and the paper's printed constants.
CPU only."""
import math
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy.optimize import minimize_scalar

from oracle import dm, net, sp2
from paper_2101_06385_amd import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.txt")


def golden():
    out = {}
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        name, value, _cite = line.split()
        out[name] = float(value)
    return out


# ----------------------------------------------------------------------------- bounds
def test_gershgorin_encloses_spectrum():
    for seed in range(3):
        w = wl.gapped(100 + seed, 80, 30)
        lo, hi = sp2.gershgorin(w.h)
        ev = np.linalg.eigvalsh(w.h)
        assert lo <= ev[0] and ev[-1] <= hi


def test_gershgorin_diagonal_is_tight():
    h = np.diag([-3.0, 1.5, 9.25, 0.0])
    lo, hi = sp2.gershgorin(h)
    assert lo <= -3.0 and abs(lo + 3.0) < 1e-13
    assert hi >= 9.25 and abs(hi - 9.25) < 1e-13


def test_rescale_reverses_and_maps_to_unit_interval():
    w = wl.gapped(4, 30, 10)
    e1, en = float(w.eps[0]), float(w.eps[-1])
    s0 = sp2.rescale(w.h, e1, en)
    lam = np.sort(np.linalg.eigvalsh(s0))
    # lowest energy -> 1, highest -> 0, linear in between
    expect = np.sort((en - w.eps) / (en - e1))
    assert np.abs(lam - expect).max() < 1e-13
    assert abs(lam[0]) < 1e-13 and abs(lam[-1] - 1.0) < 1e-13


# ----------------------------------------------------------------------------- constants
def test_theorem_constant_is_the_ratio_maximum():
    """Appendix: C is the maximum over (0,1) of both two-step ratios; Alg. 1 uses 4.5 > C."""
    g = golden()

    def r1(x):
        y = 2 * x - x * x
        return (y * y - y ** 4) / (x - x * x) ** 2

    def r2(x):
        y = 2 * x * x - x ** 4
        return (y - y * y) / (x - x * x) ** 2

    c = sp2.theorem_constant()
    for r in (r1, r2):
        grid = np.linspace(1e-4, 1 - 1e-4, 200001)
        m0 = float(np.max(r(grid)))
        best = minimize_scalar(lambda x: -r(x), bounds=(1e-6, 1 - 1e-6), method="bounded",
                               options={"xatol": 1e-12})
        assert abs(-best.fun - c) < 1e-9
        assert m0 <= c + 1e-12
    assert abs(c - g["theorem_C_approx"]) < 0.005
    assert sp2.STOP_FACTOR == g["stop_factor"] > c


def test_polynomial_order_doubles():
    """Sec. SP2 polynomials: the order doubles each step; 30 steps exceed 10^9."""
    g = golden()
    lam0 = np.linspace(0.0, 1.0, 33)
    res = sp2.sp2_eigen(lam0, 11, max_layers=6)
    p = np.polynomial.Polynomial([0.0, 1.0])
    for s in res.sigma[:6]:
        p = p * p if s > 0 else 2 * p - p * p
    assert p.degree() == 2 ** 6
    assert 2 ** int(g["steps_for_order_1e9"]) > g["order_lower_bound"]


def test_polynomial_composition_matches_recursion():
    lam0 = np.linspace(0.0, 1.0, 41)
    full = sp2.sp2_eigen(lam0, 13, max_layers=100)
    k = min(5, full.layers - 1)
    p = np.polynomial.Polynomial([0.0, 1.0])
    lam = lam0.copy()
    for s in full.sigma[:k]:
        p = p * p if s > 0 else 2 * p - p * p
        lam = lam * lam if s > 0 else 2 * lam - lam * lam
    assert np.abs(p(lam0) - lam).max() < 1e-12


# ----------------------------------------------------------------------------- Alg. 1 in FP64
def test_sp2_fp64_config1_matches_exact():
    w = wl.config1()
    res = sp2.sp2_alg1(w.h, w.n_occ)
    d_ref = dm.dm_construct(w.q, w.eps, w.n_occ)
    assert res.converged
    assert np.linalg.norm(res.d - d_ref) < 1e-10
    assert abs(np.trace(res.d) - w.n_occ) < 1e-10
    assert abs(np.trace(res.d) - np.sum(res.d * res.d)) < 1e-12   # Tr[D - D^2] (config tol)
    assert 20 <= res.layers <= 60


def test_sp2_fp64_matches_eigenvalue_recursion():
    """Alg. 1 on the matrix and on the eigenvalues of S_0 give the same layer history."""
    w = wl.gapped(7, 120, 40)
    e1, en = sp2.gershgorin(w.h)
    mres = sp2.sp2_alg1(w.h, w.n_occ, bounds=(e1, en))
    lam0 = (en - w.eps) / (en - e1)
    sres = sp2.sp2_eigen(lam0, w.n_occ)
    assert mres.layers == sres.layers
    assert mres.sigma == sres.sigma
    for a, b in zip(mres.iderr, sres.iderr):
        if abs(b) > 1e-8:
            assert abs(a - b) <= 1e-9 * max(1.0, abs(b))
    ev = np.sort(np.linalg.eigvalsh(mres.d))
    assert np.abs(ev - np.sort(sres.d)).max() < 1e-10


def test_theorem_inequality_holds_on_histories():
    """Appendix theorem: IdErr_{i+1} <= C IdErr_{i-1}^2 whenever sigma_i != sigma_{i-1}."""
    c = sp2.theorem_constant()
    checked = 0
    for seed in range(6):
        rng = np.random.default_rng(seed)
        lam0 = rng.uniform(0, 1, size=200)
        res = sp2.sp2_eigen(lam0, int(rng.integers(20, 180)))
        e = [None] + res.iderr          # 1-based
        s = [0] + res.sigma
        for i in range(2, len(e) - 1):
            if s[i] != s[i - 1] and e[i - 1] > 1e-6:
                assert e[i + 1] <= c * e[i - 1] ** 2 * (1 + 1e-9) + 1e-12
                checked += 1
    assert checked > 20


@pytest.mark.parametrize("n_occ", [0, 24])
def test_sp2_fp64_empty_and_full_occupation(n_occ):
    w = wl.gapped(8, 24, 12)
    res = sp2.sp2_alg1(w.h, n_occ)
    expect = np.zeros((24, 24)) if n_occ == 0 else np.eye(24)
    assert np.abs(res.d - expect).max() < 1e-9


def test_sp2_fp64_not_converged_when_layer_cap_is_small():
    w = wl.config1()
    res = sp2.sp2_alg1(w.h, w.n_occ, max_layers=5)
    assert not res.converged and res.layers == 5
    assert abs(np.trace(res.d) - w.n_occ) > 1e-6 or np.abs(res.d @ res.d - res.d).max() > 1e-6


def test_small_random_case_mixed_precision_and_refinement():
    """The paper's 10x10 case (H_ij in [-1,1], N_occ = 5): mixed-precision SP2 converges
    and the FP64 refinement layer improves idempotency by orders of magnitude."""
    w = wl.small_random()
    d_ref = dm.dm_eigh(w.h, w.n_occ)
    for fmt, s in (("fp16", 0), ("fp16", 12), ("bf16", 0)):
        res = sp2.sp2_alg1(w.h, w.n_occ, activation=sp2.mixed_square_fp32(fmt, s))
        assert res.converged
        sl = res.s_last
        err_before = np.linalg.norm(sl @ sl - sl, 2)
        err_after = np.linalg.norm(res.d @ res.d - res.d, 2)
        assert err_after < 1e-2 * err_before
        assert np.linalg.norm(res.d - d_ref) < 1e-3


# ----------------------------------------------------------------------------- Alg. 2
def test_round_bf16_brute_force():
    # values on and between bfloat16 grid points near 1 (spacing 2^-7)
    one = np.float32(1.0)
    cases = {
        1.0: 1.0,
        1.0 + 2 ** -8: 1.0,                    # tie -> even (1.0)
        1.0 + 3 * 2 ** -8: 1.0 + 2 ** -6,      # tie -> even (1 + 2^-6)
        1.0 + 2 ** -8 + 2 ** -20: 1.0 + 2 ** -7,
        -2.0 - 2 ** -7 - 2 ** -10: -2.0 - 2 ** -6,  # past the midpoint of [-2-2^-6, -2]
    }
    for x, want in cases.items():
        got = float(sp2.round_bf16(np.array([x], dtype=np.float32))[0])
        assert got == want, (x, got, want)
    assert float(sp2.round_bf16(np.array([one]))[0]) == 1.0


def test_split_reproduces_single_precision():
    rng = np.random.default_rng(1)
    x = rng.uniform(-1, 1, size=(40, 40)).astype(np.float32)
    x = x[np.abs(x) > 1e-3].reshape(-1)
    # 11 + 11 significant bits while the low plane stays out of the FP16 subnormal range
    # (|x| >= 1/4 unscaled; every |x| >= 1e-3 once shifted by 2^12)
    for s, lo in ((0, 0.25), (12, 1e-3)):
        xs = x[np.abs(x) >= lo]
        x0, x1 = sp2.split_planes(xs, "fp16", s)
        rec = (x0.astype(np.float64) + x1.astype(np.float64)) * 2.0 ** -s
        assert np.all(np.abs(rec - xs) <= 2.0 ** -22 * np.abs(xs))
    x0, x1 = sp2.split_planes(x, "bf16", 0)
    rec = x0.astype(np.float64) + x1.astype(np.float64)
    assert np.all(np.abs(rec - x) <= 2.0 ** -16 * np.abs(x))


def test_lo_scaling_keeps_low_plane_normal():
    """Entries ~5e-3 (converged N=8192 off-diagonals): unscaled low plane is FP16-subnormal."""
    x = np.full(5, 5.1e-3, dtype=np.float32) + np.arange(5, dtype=np.float32) * 1e-7
    _, x1 = sp2.split_planes(x, "fp16", 0)
    assert np.all(np.abs(x1[x1 != 0]) < 2.0 ** -14)
    x0s, x1s = sp2.split_planes(x, "fp16", 12)
    err0 = np.abs(sp2.split_planes(x, "fp16", 0)[0] + x1 - x)
    err12 = np.abs((x0s + x1s) * 2.0 ** -12 - x)
    assert np.all(err12 <= err0)


def test_mixed_square_brute_force_rational():
    """Small matrices of half-representable values: every term is exact, compare with Fractions."""
    rng = np.random.default_rng(2)
    n = 6
    a = rng.uniform(-1, 1, size=(n, n)).astype(np.float32)
    a = (a + a.T) / 2
    got = sp2.mixed_square(a, "fp16", 0)
    x0, x1 = sp2.split_planes(a, "fp16", 0)
    F = [[Fraction(float(v)) for v in row] for row in x0]
    G = [[Fraction(float(v)) for v in row] for row in x1]
    for i in range(n):
        for j in range(n):
            exact = sum(F[i][k] * F[k][j] + F[i][k] * G[k][j] + G[i][k] * F[k][j] for k in range(n))
            assert abs(float(exact) - got[i, j]) <= 1e-15 * max(1.0, abs(float(exact)))
    assert np.array_equal(got, got.T)


def test_mixed_square_rows_match_full_product():
    w = wl.gapped(13, 90, 30)
    x = sp2.rescale(w.h, *sp2.gershgorin(w.h)).astype(np.float32)
    rows = [0, 17, 89]
    for fmt, s in (("fp16", 12), ("bf16", 0)):
        assert np.abs(sp2.mixed_square_rows(x, rows, fmt, s) - sp2.mixed_square(x, fmt, s)[rows]).max() < 1e-15


def test_mixed_square_exact_for_half_representable_input():
    rng = np.random.default_rng(4)
    a = rng.integers(-8, 9, size=(16, 16)).astype(np.float32) / 16
    a = np.triu(a) + np.triu(a, 1).T
    assert np.array_equal(sp2.mixed_square(a, "fp16", 0), a.astype(np.float64) @ a)
    assert np.array_equal(sp2.mixed_square(a, "bf16", 0), a.astype(np.float64) @ a)


def test_mixed_square_error_is_the_dropped_term():
    rng = np.random.default_rng(5)
    w = wl.gapped(5, 64, 20)
    s0 = sp2.rescale(w.h, *sp2.gershgorin(w.h)).astype(np.float32)
    x0, x1 = sp2.split_planes(s0, "fp16", 0)
    # the planes represent xr = X0 + X1 exactly; the only product left out is X1 X1
    xr = x0.astype(np.float64) + x1.astype(np.float64)
    got = sp2.mixed_square(s0, "fp16", 0)
    dropped = x1.astype(np.float64) @ x1.astype(np.float64)
    assert np.abs(got + dropped - xr @ xr).max() < 1e-15
    # and the split itself is within 2^-22 of the FP32 input where the low plane is normal
    assert np.linalg.norm(got - s0.astype(np.float64) @ s0) < 1e-5


# ----------------------------------------------------------------------------- refinement
def test_refinement_is_two_composed_layers():
    """Sec. on convergence: f_final composes two SP2 layers with opposite signs."""
    w = wl.gapped(6, 40, 15)
    s = sp2.rescale(w.h, *sp2.gershgorin(w.h))
    for first in (1, -1):
        wts, bs, cs = net.sp2_branch_coefficients([first, -first])
        two = net.forward_matrix(s, wts, bs, cs)[-1]
        assert np.abs(sp2.refinement(s, first) - two).max() < 1e-13


def test_refinement_quadratic_gain_and_fixed_points():
    for first in (1, -1):
        z = sp2.refinement(np.diag([0.0, 1.0]), first)
        assert np.array_equal(z, np.diag([0.0, 1.0]))
        for delta in (1e-3, 1e-4):
            lo = sp2.refinement(np.diag([delta]), first)[0, 0]
            hi = 1.0 - sp2.refinement(np.diag([1.0 - delta]), first)[0, 0]
            assert lo <= 4.0001 * delta ** 2 and hi <= 4.0001 * delta ** 2


def test_network_with_sp2_coefficients_reproduces_alg1_chain():
    w = wl.gapped(12, 50, 18)
    res = sp2.sp2_alg1(w.h, w.n_occ)
    s0 = sp2.rescale(w.h, *res.bounds)
    wts, bs, cs = net.sp2_branch_coefficients(res.sigma[: res.layers - 1])
    chain = net.forward_matrix(s0, wts, bs, cs)[-1]
    assert np.abs(chain - res.s_last).max() < 1e-12
