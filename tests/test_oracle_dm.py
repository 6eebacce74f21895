"""Pins of the exact density-matrix oracle (Eqs. 1, 3-6) against closed forms,
invariants and brute force.  CPU only."""
import numpy as np
import pytest

from oracle import dm
from paper_2101_06385_amd import workloads as wl


def _invariants(h, d, n_occ, tol):
    n = h.shape[0]
    assert np.abs(d - d.T).max() < tol
    assert np.abs(d @ d - d).max() < tol                       # idempotent
    assert abs(np.trace(d) - n_occ) < tol * n                  # occupation
    assert np.abs(h @ d - d @ h).max() < tol * np.abs(h).max() * n  # commutes with H
    ev = np.linalg.eigvalsh(d)
    assert np.all(np.minimum(np.abs(ev), np.abs(ev - 1.0)) < tol)  # eigenvalues in {0,1}


def test_eigh_matches_construction_config1():
    w = wl.config1()
    d1 = dm.dm_eigh(w.h, w.n_occ)
    d2 = dm.dm_construct(w.q, w.eps, w.n_occ)
    assert np.linalg.norm(d1 - d2) < 1e-11
    _invariants(w.h, d1, w.n_occ, 1e-11)


@pytest.mark.parametrize("n,n_occ", [(1, 0), (1, 1), (7, 3), (64, 17), (96, 96), (96, 0)])
def test_eigh_matches_construction_small(n, n_occ):
    w = wl.gapped(11 + n, n, n_occ)
    d1 = dm.dm_eigh(w.h, n_occ)
    d2 = dm.dm_construct(w.q, w.eps, n_occ)
    assert np.linalg.norm(d1 - d2) < 1e-11
    _invariants(w.h, d1, n_occ, 1e-11)


def test_one_by_one():
    h = np.array([[3.7]])
    assert dm.dm_eigh(h, 0)[0, 0] == 0.0
    assert abs(dm.dm_eigh(h, 1)[0, 0] - 1.0) < 1e-15


def test_two_by_two_closed_form():
    a, b, c = 0.3, -1.1, 2.0
    h = np.array([[a, b], [b, c]])
    lam = 0.5 * (a + c) - np.sqrt((0.5 * (a - c)) ** 2 + b * b)
    # eigenvector of the lower eigenvalue, by hand: (b, lam - a)
    v = np.array([b, lam - a])
    v /= np.linalg.norm(v)
    d = dm.dm_eigh(h, 1)
    assert np.abs(d - np.outer(v, v)).max() < 1e-14


def test_diagonal_reduces_to_sorting():
    rng = np.random.default_rng(3)
    vals = rng.permutation(np.arange(12, dtype=float) * 1.5 - 4.0)
    h = np.diag(vals)
    n_occ = 5
    d = dm.dm_eigh(h, n_occ)
    lowest = np.argsort(vals)[:n_occ]
    expect = np.zeros(12)
    expect[lowest] = 1.0
    assert np.abs(d - np.diag(expect)).max() < 1e-15


def test_particle_hole_shift_scale_permutation():
    w = wl.gapped(5, 48, 20)
    d = dm.dm_eigh(w.h, 20)
    n = w.n
    # particle-hole: D(-H, N - N_occ) = I - D(H, N_occ)
    assert np.abs(dm.dm_eigh(-w.h, n - 20) - (np.eye(n) - d)).max() < 1e-11
    # shift and positive scale leave D unchanged
    assert np.abs(dm.dm_eigh(2.5 * w.h + 7.0 * np.eye(n), 20) - d).max() < 1e-11
    # permutation covariance: D(P H P^T) = P D P^T
    p = np.random.default_rng(9).permutation(n)
    pm = np.eye(n)[p]
    assert np.abs(dm.dm_eigh(pm @ w.h @ pm.T, 20) - pm @ d @ pm.T).max() < 1e-11


def test_fermi_dirac_properties():
    x = np.linspace(-3, 3, 61)
    f = dm.fermi_dirac(x, 0.0, 0.2)
    assert abs(dm.fermi_dirac(np.array([0.7]), 0.7, 0.1)[0] - 0.5) < 1e-15
    assert np.abs(f + f[::-1] - 1.0).max() < 1e-15             # f(mu+x) + f(mu-x) = 1
    assert np.all(np.diff(f) <= 0)
    # zero-temperature limit: the projector, for a gapped spectrum with mu in the gap
    w = wl.gapped(21, 40, 12)
    mu = 0.5 * (w.homo + w.lumo)
    assert np.abs(dm.dm_fermi(w.q, w.eps, mu, 1e-3) - dm.dm_construct(w.q, w.eps, 12)).max() < 1e-12
    # rescaled Fermi function of Eq. fermi: F(1/2) = 1/2, F(0) = 1/(e^-20 + 1)
    assert abs(dm.fermi_rescaled(np.array([0.5]))[0] - 0.5) < 1e-15
    assert abs(dm.fermi_rescaled(np.array([0.0]))[0] - 1.0 / (np.exp(-20.0) + 1.0)) < 1e-15


def test_dm_rows_matches_full():
    w = wl.gapped(2, 50, 21)
    rows = [0, 7, 49]
    assert np.abs(dm.dm_rows(w.q, w.eps, 21, rows) - dm.dm_construct(w.q, w.eps, 21)[rows]).max() < 1e-15
