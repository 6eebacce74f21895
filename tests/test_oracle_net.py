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


def test_perturbed_chain_without_perturbation_is_the_plain_chain():
    _, _, lam0, _, tvals, wt, bt, ct = _problem(n=100, k=6, seed=2)
    l0, w0, b0, c0, _ = net.loss_grad_scalar(lam0, tvals, wt, bt, ct)
    l1, w1, b1, c1, _ = net.loss_grad_scalar_perturbed(lam0, tvals, wt, bt, ct)
    assert l0 == l1 and np.array_equal(w0, w1) and np.array_equal(b0, b1) and np.array_equal(c0, c1)


def test_perturbed_chain_at_the_last_layer_shifts_the_output():
    """A shift d after the last layer changes the loss by exactly 2 d sum(x_K - t) + N d^2
    (the closed form of a shifted sum of squares)."""
    _, _, lam0, _, tvals, wt, bt, ct = _problem(n=100, k=6, seed=3)
    l0, *_ = net.loss_grad_scalar(lam0, tvals, wt, bt, ct)
    xk = net.forward_scalar(lam0, wt, bt, ct)[-1]
    d = 1e-3
    l1, *_ = net.loss_grad_scalar_perturbed(lam0, tvals, wt, bt, ct, layer=5, delta=d)
    want = l0 + 2 * d * np.sum(xk - tvals) + len(lam0) * d * d
    assert abs(l1 - want) < 1e-10 * max(1.0, abs(want))


def test_gradient_error_bound_is_linear_and_covers_random_perturbations():
    """The bound is zero for error-free layers, scales linearly at small errors, and covers
    the gradient change of a random-sign perturbation of the same size at every layer."""
    _, _, lam0, _, tvals, wt, bt, ct = _problem(n=300, k=8, seed=4)
    z = net.gradient_error_bound(lam0, tvals, wt, bt, ct, 0.0)
    assert all(np.all(a == 0) for a in z)
    b1 = np.concatenate(net.gradient_error_bound(lam0, tvals, wt, bt, ct, 1e-7))
    b2 = np.concatenate(net.gradient_error_bound(lam0, tvals, wt, bt, ct, 2e-7))
    assert np.allclose(b2, 2 * b1, rtol=1e-3, atol=1e-12)
    # random signs per eigenvalue and layer, magnitude 1e-7 max|x_{k+1}|
    rng = np.random.default_rng(5)
    xs = [lam0]
    for k in range(len(wt)):
        y = wt[k] * xs[-1] ** 2 + bt[k] * xs[-1] + ct[k]
        xs.append(y + 1e-7 * np.abs(y).max() * rng.choice([-1.0, 1.0], size=len(y)))
    g = 2.0 * (xs[-1] - tvals)
    got = []
    for k in range(len(wt) - 1, -1, -1):
        x = xs[k]
        got.append((np.sum(g * x * x), np.sum(g * x), np.sum(g)))
        g = g * (2.0 * wt[k] * x + bt[k])
    got = np.array(got[::-1]).T.reshape(-1)
    _, w0, b0, c0, _ = net.loss_grad_scalar(lam0, tvals, wt, bt, ct)
    ref = np.concatenate([w0, b0, c0])
    assert np.all(np.abs(got - ref) <= b1 * 1.01 + 1e-12)


def test_adam_first_step_closed_form():
    """With zero moments the bias-corrected first step is -lr g / (|g| + eps) per
    coefficient: each one moves by lr against the sign of its gradient."""
    _, _, lam0, _, tvals, wt, bt, ct = _problem(n=80, k=5, seed=6)
    _, dw, db, dc = net.loss_grad_scalar(lam0, tvals, wt, bt, ct)[:4]
    lr = 1e-3
    _, w1, b1, c1 = net.adam_scalar(lam0, tvals, wt, bt, ct, lr, 1)
    g = np.concatenate([dw, db, dc])
    moved = np.concatenate([w1 - wt, b1 - bt, c1 - ct])
    assert np.allclose(moved, -lr * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)


def test_adam_matches_a_library_adam():
    """30 steps of the oracle's Adam against torch.optim.Adam in FP64 on the CPU (an
    independent implementation of the same published method) with the same gradients."""
    import torch

    _, _, lam0, _, tvals, wt, bt, ct = _problem(n=120, k=6, seed=7)
    lr, steps = 2e-3, 30
    losses, w1, b1, c1 = net.adam_scalar(lam0, tvals, wt, bt, ct, lr, steps)
    p = torch.tensor(np.concatenate([wt, bt, ct]), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([p], lr=lr)
    k = len(wt)
    tl = []
    for _ in range(steps):
        pn = p.detach().numpy()
        loss, dw, db, dc, _ = net.loss_grad_scalar(lam0, tvals, pn[:k], pn[k:2 * k], pn[2 * k:])
        tl.append(loss)
        opt.zero_grad()
        p.grad = torch.tensor(np.concatenate([dw, db, dc]), dtype=torch.float64)
        opt.step()
    pn = p.detach().numpy()
    assert np.allclose(losses, tl, rtol=1e-10)
    assert np.allclose(np.concatenate([w1, b1, c1]), pn, rtol=1e-10, atol=1e-13)


def test_adam_fit_lowers_the_config5_loss():
    """The fit the GPU network runs (truncated SP2 start, lr 3e-3): on the C5 spectrum at
    n = 512 the eigenvalue loss falls well below its start in 150 steps."""
    w = wl.config5(seed=5000, n=512)
    e1, en = sp2.gershgorin(w.h)
    lam0 = (en - w.eps) / (en - e1)
    tvals = dm.fermi_dirac(w.eps, 0.0, 0.2)
    k = 20
    sig = (list(sp2.sp2_eigen(lam0, 256, max_layers=k).sigma) + [1, -1] * k)[:k]
    wt, bt, ct = net.sp2_branch_coefficients(sig)
    losses, *_ = net.adam_scalar(lam0, tvals, wt, bt, ct, 3e-3, 150)
    assert np.all(np.isfinite(losses))
    assert losses[-1] < 0.6 * losses[0], (losses[0], losses[-1])
