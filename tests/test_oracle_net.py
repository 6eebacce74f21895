"""Pins of the network oracle (Eq. general SP2, squared-error loss): matrix vs eigenvalue
recursion, hand-derived gradient vs central finite differences (h = 1e-4, FP64).  CPU only."""
import numpy as np

from oracle import dm, net, sp2
from paper_2101_06385_amd import workloads as wl


def _problem(n=64, k=8, seed=0):
    w = wl.config5(seed=seed, n=n)
    e1, en = sp2.gershgorin(w.h)
    x0 = sp2.rescale(w.h, e1, en)
    lam0 = (en - w.eps) / (en - e1)
    target = dm.dm_fermi(w.q, w.eps, 0.0, 0.2)
    tvals = dm.fermi_dirac(w.eps, 0.0, 0.2)
    rng = np.random.default_rng(seed)
    sig = rng.choice([-1, 1], size=k)
    wt, bt, ct = net.sp2_branch_coefficients(sig)
    wt = wt + rng.normal(0, 0.05, k)
    bt = bt + rng.normal(0, 0.05, k)
    ct = ct + rng.normal(0, 0.01, k)
    return w, x0, lam0, target, tvals, wt, bt, ct


def test_matrix_forward_is_eigenvalue_forward():
    w, x0, lam0, _, _, wt, bt, ct = _problem()
    xk = net.forward_matrix(x0, wt, bt, ct)[-1]
    lk = net.forward_scalar(lam0, wt, bt, ct)[-1]
    assert np.abs(xk - (w.q * lk[None, :]) @ w.q.T).max() < 1e-10


def test_loss_matrix_equals_eigenvalue_loss():
    w, x0, lam0, target, tvals, wt, bt, ct = _problem()
    lm = net.loss_grad_matrix(x0, target, wt, bt, ct)[0]
    ls = net.loss_scalar(lam0, tvals, wt, bt, ct)
    assert abs(lm - ls) < 1e-9 * max(1.0, ls)


def test_scalar_gradient_matches_finite_differences():
    _, _, lam0, _, tvals, wt, bt, ct = _problem(n=200, k=10, seed=1)
    _, dw, db, dc, _ = net.loss_grad_scalar(lam0, tvals, wt, bt, ct)
    fw, fb, fc = net.finite_difference_grad(lam0, tvals, wt, bt, ct, h=1e-4)
    for a, b in ((dw, fw), (db, fb), (dc, fc)):
        assert np.abs(a - b).max() <= 1e-5 * max(1.0, np.abs(b).max())


def test_matrix_adjoint_matches_scalar_gradient():
    _, x0, lam0, target, tvals, wt, bt, ct = _problem(n=64, k=8, seed=2)
    _, mw, mb, mc, _ = net.loss_grad_matrix(x0, target, wt, bt, ct)
    _, sw, sb, sc, _ = net.loss_grad_scalar(lam0, tvals, wt, bt, ct)
    for a, b in ((mw, sw), (mb, sb), (mc, sc)):
        assert np.abs(a - b).max() <= 1e-8 * max(1.0, np.abs(b).max())


def test_matrix_adjoint_input_gradient_by_directional_difference():
    _, x0, _, target, _, wt, bt, ct = _problem(n=24, k=5, seed=3)
    _, _, _, _, g0 = net.loss_grad_matrix(x0, target, wt, bt, ct)
    rng = np.random.default_rng(7)
    v = rng.normal(size=x0.shape)
    v = 0.5 * (v + v.T)
    h = 1e-5

    def loss(x):
        return net.loss_grad_matrix(x, target, wt, bt, ct)[0]

    fd = (loss(x0 + h * v) - loss(x0 - h * v)) / (2 * h)
    assert abs(fd - float(np.sum(g0 * v))) <= 1e-6 * max(1.0, abs(fd))
