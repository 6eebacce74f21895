"""Parity of the finite-temperature expansion on matrices (sp2_fermi_apply through the C
ABI) against the oracle: every X_k is a polynomial in H, so the exact result of the
network is Q diag(F~(x)) Q^T with x the rescaled spectrum (pinned in the oracle tests).

Bars: FP64 1e-10 elementwise; FP32 state modes (FP32, FP16X2, BF16X2) 1e-3 sqrt(N) in the
Frobenius norm, as for the density matrix, and 1e-4 elementwise for FP32/FP16X2.
"""
import numpy as np
import pytest
import torch

from oracle import fermi as f
from oracle import sp2 as osp2
from paper_2101_06385_amd import sp2, workloads as wl

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _exact(w, theta, c, bounds, rows=None):
    x = (w.eps - bounds[0]) / (bounds[1] - bounds[0])
    vals = f.model_scalar(x, theta, c)
    q = w.q if rows is None else w.q[rows]
    return (q * vals[None, :]) @ w.q.T, vals


def _case(n, seed=101):
    rng = np.random.default_rng(seed)
    eps = np.sort(rng.uniform(-15.0, 15.0, n))
    return wl._build("fermi_n%d" % n, rng, eps, n // 2, float("nan"), float("nan"))


@pytest.mark.parametrize("prec,tol_max", [("fp64", 1e-10), ("fp32", 1e-4), ("fp16x2", 1e-4), ("bf16x2", 3e-3)])
def test_fermi_apply_matches_eigenbasis(prec, tol_max):
    w = _case(700)
    bounds = (-15.5, 15.5)
    theta, c, _ = sp2.fermi_fit(11, 0.0, 0.2, bounds)
    h = torch.from_numpy(w.h).to(DEV)
    d, obs = sp2.fermi_apply(h, theta, c, bounds, precision=prec)
    d = d.cpu().numpy()
    ref, vals = _exact(w, theta, c, bounds)
    err = np.abs(d - ref).max()
    print("%s: max |D - D_ref| = %.3e, Frobenius %.3e" % (prec, err, np.linalg.norm(d - ref)))
    assert err <= tol_max
    assert np.linalg.norm(d - ref) <= 1e-3 * np.sqrt(w.n)
    assert np.array_equal(d, d.T)
    assert abs(obs[0] - vals.sum()) <= max(1e-9, 10 * tol_max) * w.n
    assert abs(obs[1] - (vals ** 2).sum()) <= max(1e-9, 10 * tol_max) * w.n
    assert abs(obs[2] - (vals * w.eps).sum()) <= max(1e-9, 10 * tol_max) * 15.0 * w.n


def test_fermi_apply_fp64_against_matrix_oracle_and_fermi():
    """FP64: the oracle's matrix recursion and, through the fit error, the exact Fermi
    operator Q diag(F(e)) Q^T."""
    w = _case(300, seed=102)
    bounds = (-16.0, 15.0)
    theta, c, loss = sp2.fermi_fit(11, 0.0, 0.2, bounds)
    h = torch.from_numpy(w.h).to(DEV)
    d, _ = sp2.fermi_apply(h, theta, c, bounds, precision="fp64")
    d = d.cpu().numpy()
    assert np.abs(d - f.model_matrix(w.h, theta, c, *bounds)).max() < 1e-10
    x = (w.eps - bounds[0]) / (bounds[1] - bounds[0])
    fit_err = np.abs(f.model_scalar(x, theta, c) - f.fermi(x, (bounds[1] - bounds[0]) / 0.2,
                                                           (0.0 - bounds[0]) / (bounds[1] - bounds[0]))).max()
    exact = (w.q * (1.0 / (np.exp(w.eps / 0.2) + 1.0))[None, :]) @ w.q.T
    assert np.abs(d - exact).max() <= fit_err * 1.01 + 1e-10


@pytest.mark.parametrize("n", [1, 2, 65, 129])
def test_fermi_apply_small_and_ragged(n):
    w = _case(n, seed=103 + n)
    bounds = (-15.0, 15.0)
    theta, c, _ = sp2.fermi_fit(4, 0.0, 1.0, bounds)
    h = torch.from_numpy(w.h).to(DEV)
    for prec, tol in (("fp64", 1e-11), ("fp16x2", 1e-4)):
        d, _ = sp2.fermi_apply(h, theta, c, bounds, precision=prec)
        ref, _ = _exact(w, theta, c, bounds)
        assert np.abs(d.cpu().numpy() - ref).max() <= tol, (n, prec)


def test_fermi_apply_leading_dimensions_and_one_layer():
    w = _case(200, seed=104)
    bounds = (-15.0, 15.0)
    theta, c, _ = sp2.fermi_fit(1, 0.0, 3.0, bounds)
    big = torch.zeros((200, 256), dtype=torch.float64, device=DEV)
    big[:, :200] = torch.from_numpy(w.h).to(DEV)
    hv = big[:, :200]
    out = torch.full((200, 230), 7.0, dtype=torch.float64, device=DEV)
    sp2.fermi_apply(hv, theta, c, bounds, precision="fp64", out=out[:, :200])
    ref, _ = _exact(w, theta, c, bounds)
    o = out.cpu().numpy()
    assert np.abs(o[:, :200] - ref).max() < 1e-12
    assert np.all(o[:, 200:] == 7.0)


def test_fermi_apply_argument_errors():
    w = _case(50, seed=105)
    h = torch.from_numpy(w.h).to(DEV)
    theta, c, _ = sp2.fermi_fit(3, 0.0, 1.0, (-15.0, 15.0))
    c_bad = c.copy()
    c_bad[1] = np.nan
    with pytest.raises(sp2.SP2Error):
        sp2.fermi_apply(h, theta, c_bad, (-15.0, 15.0))
    with pytest.raises(ValueError):
        sp2.fermi_apply(h, theta, c[:-1], (-15.0, 15.0))
    with pytest.raises(sp2.SP2Error):
        sp2.fermi_apply(h, theta, c, (1.0, -1.0))


def test_spectral_bounds_match_oracle():
    w = _case(333, seed=106)
    lo, hi = sp2.spectral_bounds(torch.from_numpy(w.h).to(DEV))
    rlo, rhi = osp2.gershgorin(w.h)
    assert abs(lo - rlo) <= 1e-12 * abs(rlo) and abs(hi - rhi) <= 1e-12 * abs(rhi)
    assert lo <= w.eps[0] and w.eps[-1] <= hi


def test_fermi_paper_case_8192_sampled_rows():
    """The section's case (11 layers, beta = 40 and mu = 1/2 in the rescaled energy) on an
    N = 8192 Hamiltonian with Gershgorin bounds, FP16X2 on the persistent kernel: sampled
    rows against Q diag(F~(x)) Q^T."""
    rng = np.random.default_rng(107)
    n = 8192
    eps = np.sort(rng.uniform(-15.0, 15.0, n))
    q = wl.haar_orthogonal(rng, n, DEV)
    hm = wl.symmetric_from_eigen(q, eps, DEV)
    h = torch.from_numpy(hm).to(DEV)
    bounds = sp2.spectral_bounds(h)
    span = bounds[1] - bounds[0]
    theta, c, _ = sp2.fermi_fit(11, bounds[0] + 0.5 * span, span / 40.0, bounds)
    d, obs = sp2.fermi_apply(h, theta, c, bounds)
    rows = [0, 4000, 8191]
    d = d.cpu().numpy()
    x = (eps - bounds[0]) / span
    vals = f.model_scalar(x, theta, c)
    ref = (q[rows] * vals[None, :]) @ q.T
    assert np.abs(d[rows] - ref).max() <= 1e-4
    assert np.array_equal(d[rows][:, :64], d[:64][:, rows].T)
    assert abs(obs[0] - np.trace(d)) <= 1e-9 * n
    # Eq. Square drops X1 X1: each FP16X2 layer biases the trace by up to 2^-24 ||X_k||_F^2
    # <= 2^-24 N (|theta_k1| <= 2 here), and the layers after it scale that by at most the
    # network's slope (beta/4 = 10 at mu); the network has no trace correction
    assert np.abs(theta[:, 0]).max() <= 2.5
    assert abs(obs[0] - vals.sum()) <= 11 * 2.5 * 2.0 ** -24 * n * 10
