"""Parity of the differentiable generalized-SP2 network (Eq. general SP2 on matrices)
against the CPU oracle: forward layers, the hand-written adjoint (dW, dB, dc and dL/dX_0),
checkpoint recomputation, and the autograd wrapper."""
import numpy as np
import pytest
import torch

from oracle import dm, net as onet, sp2 as osp2
from paper_2101_06385_amd import net as gnet, sp2, workloads as wl

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _problem(n, k, seed, spread=0.02):
    w = wl.config5(seed=seed, n=n)
    e1, en = osp2.gershgorin(w.h)
    x0 = osp2.rescale(w.h, e1, en).astype(np.float32)       # the input layer S_0, as FP32
    lam0 = (en - w.eps) / (en - e1)
    sig = osp2.sp2_eigen(lam0, n // 2, max_layers=k).sigma
    sig = (sig + [1, -1] * k)[:k]
    wt, bt, ct = onet.sp2_branch_coefficients(sig)
    rng = np.random.default_rng(seed)
    wt = (wt + rng.normal(0, spread, k)).astype(np.float32)
    bt = (bt + rng.normal(0, spread, k)).astype(np.float32)
    ct = (ct + rng.normal(0, spread / 4, k)).astype(np.float32)
    target = dm.dm_fermi(w.q, w.eps, 0.0, 0.2)
    return w, x0, wt, bt, ct, target


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


@pytest.mark.parametrize("prec,n,k", [("fp32", 200, 6), ("fp16x2", 200, 6), ("bf16x2", 130, 4), ("fp16x2", 520, 10)])
def test_forward_matches_fp64_layers(prec, n, k):
    w, x0, wt, bt, ct, _ = _problem(n, k, 10 + n)
    xk, _ = sp2.net_forward(_t(x0), _t(wt), _t(bt), _t(ct), precision=prec)
    ref = onet.forward_matrix(x0.astype(np.float64), wt.astype(np.float64), bt.astype(np.float64),
                              ct.astype(np.float64))[-1]
    got = xk.cpu().numpy().astype(np.float64)
    tol = {"fp32": 2e-5, "fp16x2": 2e-4, "bf16x2": 2e-3}[prec]
    assert np.abs(got - ref).max() <= tol * max(1.0, np.abs(ref).max()), float(np.abs(got - ref).max())
    assert np.array_equal(got, got.T)


def test_sp2_branch_coefficients_reproduce_alg1_chain():
    w = wl.gapped(12, 300, 100)
    res = osp2.sp2_alg1(w.h, w.n_occ)
    x0 = osp2.rescale(w.h, *res.bounds).astype(np.float32)
    sig = res.sigma[:12]
    wt, bt, ct = [a.astype(np.float32) for a in onet.sp2_branch_coefficients(sig)]
    xk, _ = sp2.net_forward(_t(x0), _t(wt), _t(bt), _t(ct), precision="fp32")
    ref = onet.forward_matrix(x0.astype(np.float64), *onet.sp2_branch_coefficients(sig))[-1]
    assert np.abs(xk.cpu().numpy() - ref).max() < 1e-4


@pytest.mark.parametrize("prec", ["fp32", "fp16x2"])
def test_adjoint_matches_oracle_gradient(prec):
    n, k = 256, 8
    w, x0, wt, bt, ct, target = _problem(n, k, 3)
    xt, wtt, btt, ctt = _t(x0), _t(wt), _t(bt), _t(ct)
    xk, ws = sp2.net_forward(xt, wtt, btt, ctt, precision=prec)
    gk = 2.0 * (xk.double() - _t(target)).float()
    dw, db, dc, g0 = sp2.net_backward(gk, wtt, btt, ctt, ws, precision=prec)
    loss, rw, rb, rc, rg = onet.loss_grad_matrix(x0.astype(np.float64), target, wt.astype(np.float64),
                                                 bt.astype(np.float64), ct.astype(np.float64))
    tol = 2e-4 if prec == "fp32" else 2e-3
    for got, ref in ((dw, rw), (db, rb), (dc, rc)):
        got = got.cpu().numpy().astype(np.float64)
        assert np.abs(got - ref).max() <= tol * np.abs(ref).max(), (prec, got, ref)
    g0n = g0.cpu().numpy().astype(np.float64)
    assert np.abs(g0n - rg).max() <= tol * np.abs(rg).max()


@pytest.mark.parametrize("prec,n", [("fp32", 256), ("fp16x2", 300)])
def test_backward_takes_the_symmetric_part_of_a_general_gradient(prec, n):
    """sp2_net_backward given a non-symmetric G_K (through the C ABI) returns the adjoint of
    (G_K + G_K^T)/2, the gradient with respect to the symmetric output: against the FP64 matrix
    adjoint started from that symmetric part, with a ragged edge at n = 300."""
    k = 6
    w, x0, wt, bt, ct, _ = _problem(n, k, 21 + n)
    rng = np.random.default_rng(22 + n)
    g = rng.standard_normal((n, n)).astype(np.float32)
    xt, wtt, btt, ctt = _t(x0), _t(wt), _t(bt), _t(ct)
    _, ws = sp2.net_forward(xt, wtt, btt, ctt, precision=prec)
    dw, db, dc, g0 = sp2.net_backward(_t(g), wtt, btt, ctt, ws, precision=prec)
    xs = onet.forward_matrix(x0.astype(np.float64), wt.astype(np.float64), bt.astype(np.float64),
                             ct.astype(np.float64))
    gsym = 0.5 * (g.astype(np.float64) + g.T.astype(np.float64))
    # the oracle starts its adjoint from 2 (X_K - T); this T makes that start gsym
    _, rw, rb, rc, rg = onet.loss_grad_matrix(x0.astype(np.float64), xs[-1] - 0.5 * gsym, wt.astype(np.float64),
                                              bt.astype(np.float64), ct.astype(np.float64))
    tol = 2e-4 if prec == "fp32" else 2e-3
    for got, ref in ((dw, rw), (db, rb), (dc, rc)):
        got = got.cpu().numpy().astype(np.float64)
        assert np.abs(got - ref).max() <= tol * np.abs(ref).max(), (prec, got, ref)
    g0n = g0.cpu().numpy().astype(np.float64)
    assert np.abs(g0n - rg).max() <= tol * np.abs(rg).max()
    assert np.array_equal(g0n, g0n.T)


@pytest.mark.parametrize("prec,n,k", [("fp32", 700, 5), ("fp16x2", 900, 6)])
def test_adjoint_128_tiles_matches_oracle_gradient(prec, n, k):
    """Sizes above 512 run the 128-tile adjoint and forward kernels (several tiles and a
    ragged edge): gradients and dL/dX_0 against the FP64 matrix adjoint."""
    w, x0, wt, bt, ct, target = _problem(n, k, 7)
    xt, wtt, btt, ctt = _t(x0), _t(wt), _t(bt), _t(ct)
    xk, ws = sp2.net_forward(xt, wtt, btt, ctt, precision=prec)
    gk = 2.0 * (xk.double() - _t(target)).float()
    dw, db, dc, g0 = sp2.net_backward(gk, wtt, btt, ctt, ws, precision=prec)
    loss, rw, rb, rc, rg = onet.loss_grad_matrix(x0.astype(np.float64), target, wt.astype(np.float64),
                                                 bt.astype(np.float64), ct.astype(np.float64))
    tol = 2e-4 if prec == "fp32" else 2e-3
    for got, ref in ((dw, rw), (db, rb), (dc, rc)):
        got = got.cpu().numpy().astype(np.float64)
        assert np.abs(got - ref).max() <= tol * np.abs(ref).max(), (prec, got, ref)
    g0n = g0.cpu().numpy().astype(np.float64)
    assert np.abs(g0n - rg).max() <= tol * np.abs(rg).max()
    assert np.array_equal(g0n, g0n.T)


def test_adjoint_matches_central_differences_of_the_gpu_forward():
    """FP32 layers, h = 1e-2: the GPU backward equals the slope of the GPU forward."""
    n, k = 128, 5
    w, x0, wt, bt, ct, target = _problem(n, k, 4)
    xt, tt = _t(x0), _t(target)

    def loss(wv, bv, cv):
        xk, _ = sp2.net_forward(xt, _t(wv), _t(bv), _t(cv), precision="fp32")
        return float(((xk.double() - tt) ** 2).sum())

    xk, ws = sp2.net_forward(xt, _t(wt), _t(bt), _t(ct), precision="fp32")
    dw, db, dc, _ = sp2.net_backward((2.0 * (xk.double() - tt)).float(), _t(wt), _t(bt), _t(ct), ws,
                                     precision="fp32", want_g0=False)
    h = 1e-2
    for arr_i, grad in ((0, dw), (1, db), (2, dc)):
        for j in (0, k // 2, k - 1):
            p = [wt.copy(), bt.copy(), ct.copy()]
            m = [wt.copy(), bt.copy(), ct.copy()]
            p[arr_i][j] += h
            m[arr_i][j] -= h
            fd = (loss(*p) - loss(*m)) / (2 * h)
            assert abs(fd - float(grad[j])) <= 2e-2 * max(1.0, abs(fd)), (arr_i, j, fd, float(grad[j]))


def test_checkpoint_recompute_is_bit_identical():
    n, k = 200, 9
    w, x0, wt, bt, ct, target = _problem(n, k, 5)
    outs = []
    for c in (1, 3, 9, 0):
        xk, ws = sp2.net_forward(_t(x0), _t(wt), _t(bt), _t(ct), precision="fp16x2", ckpt_every=c)
        gk = (2.0 * (xk.double() - _t(target))).float()
        outs.append([xk] + list(sp2.net_backward(gk, _t(wt), _t(bt), _t(ct), ws, precision="fp16x2",
                                                 ckpt_every=c)))
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            assert torch.equal(a, b)


def test_autograd_module_trains():
    n, k = 256, 10
    w, x0, wt, bt, ct, target = _problem(n, k, 6, spread=0.0)
    lam0 = (osp2.gershgorin(w.h)[1] - w.eps) / (osp2.gershgorin(w.h)[1] - osp2.gershgorin(w.h)[0])
    sig = osp2.sp2_eigen(lam0, n // 2, max_layers=k).sigma
    model = gnet.SP2Net((sig + [1, -1] * k)[:k], precision="fp16x2", device=DEV)
    xt, tt = _t(x0), _t(target).float()
    opt = torch.optim.Adam(model.parameters(), lr=3e-3)
    losses = []
    for _ in range(15):
        opt.zero_grad()
        loss = ((model(xt) - tt) ** 2).sum()
        loss.backward()
        opt.step()
        losses.append(float(loss))
    assert np.isfinite(losses).all()
    assert losses[-1] < 0.7 * losses[0], losses


def test_config5_full_size_loss_and_gradient():
    """N = 2048, 20 layers, kT = 0.2 eV target: the matrix loss and gradient against the
    exact eigenvalue-space loss and gradient of the same coefficients (FP64 oracle)."""
    n, k = 2048, 20
    w, x0, wt, bt, ct, target = _problem(n, k, 5000, spread=0.0)
    e1, en = osp2.gershgorin(w.h)
    lam0 = (en - w.eps) / (en - e1)
    tvals = dm.fermi_dirac(w.eps, 0.0, 0.2)
    xt = _t(x0)
    xk, ws = sp2.net_forward(xt, _t(wt), _t(bt), _t(ct), precision="fp16x2")
    diff = xk.double() - _t(target)
    loss = float((diff ** 2).sum())
    dw, db, dc, _ = sp2.net_backward((2.0 * diff).float(), _t(wt), _t(bt), _t(ct), ws, precision="fp16x2",
                                     want_g0=False)
    w64, b64, c64 = wt.astype(np.float64), bt.astype(np.float64), ct.astype(np.float64)
    rl, rw, rb, rc, _ = onet.loss_grad_scalar(lam0, tvals, w64, b64, c64)
    assert abs(loss - rl) <= 1e-3 * rl + 1e-2, (loss, rl)
    # Tolerance from the layer error bound: each FP16X2 layer output carries at most
    # 2 u16^2 (the split representation, u16 = 2^-11) plus sqrt(n) u32 (FP32 accumulation
    # over n terms, u32 = 2^-24) of max|x|; the FP32 adjoint layers another sqrt(n) u32.
    # gradient_error_bound propagates that through the rest of the chain (worst sign).
    rel = 2 * 2.0 ** -22 + 2 * np.sqrt(n) * 2.0 ** -24
    tw, tb, tc = onet.gradient_error_bound(lam0, tvals, w64, b64, c64, rel)
    for got, ref, tol in ((dw, rw, tw), (db, rb, tb), (dc, rc, tc)):
        g = got.cpu().numpy().astype(np.float64)
        print("C5 gradient: max |err| / derived bound = %.3f" % float((np.abs(g - ref) / tol).max()))
        assert np.all(np.abs(g - ref) <= tol), (g[:4], ref[:4], tol[:4])


def test_config5_fit_tracks_the_oracle():
    """The C5 fit: the N = 2048, 20-layer FP16X2 network trained with Adam (lr 3e-3, 150
    steps) on the kT = 0.2 eV target from the truncated-SP2 start, against the oracle's
    FP64 Adam on the exact eigenvalue loss from the same start.  The GPU loss stays within
    1 % of the oracle's at every step (measured: 1e-4), and the fit ends below 0.45 of the
    starting loss (both reach 0.41: 54.7 -> 22.2)."""
    n, k, lr, steps = 2048, 20, 3e-3, 150
    w = wl.config5(seed=5000, n=n)
    e1, en = osp2.gershgorin(w.h)
    x0 = osp2.rescale(w.h, e1, en).astype(np.float32)
    lam0 = (en - w.eps) / (en - e1)
    tvals = dm.fermi_dirac(w.eps, 0.0, 0.2)
    sig = (list(osp2.sp2_eigen(lam0, n // 2, max_layers=k).sigma) + [1, -1] * k)[:k]
    wt, bt, ct = onet.sp2_branch_coefficients(sig)
    ref, *_ = onet.adam_scalar(lam0, tvals, wt, bt, ct, lr, steps)
    model = gnet.SP2Net(sig, precision="fp16x2", device=DEV)
    xt = _t(x0)
    tt = _t(dm.dm_fermi(w.q, w.eps, 0.0, 0.2))
    opt = torch.optim.Adam(model.parameters(), lr=lr)
    got = []
    for _ in range(steps):
        opt.zero_grad()
        loss = ((model(xt).double() - tt) ** 2).sum()
        loss.backward()
        opt.step()
        got.append(float(loss.detach()))
    got = np.array(got)
    dev = np.abs(got - ref) / ref
    print("C5 fit: loss %.4g -> %.4g (oracle %.4g -> %.4g), max relative deviation %.4f at step %d"
          % (got[0], got[-1], ref[0], ref[-1], dev.max(), int(dev.argmax())))
    assert np.all(np.isfinite(got))
    assert abs(got[0] - ref[0]) <= 1e-3 * ref[0]
    assert dev.max() <= 0.01
    assert got[-1] < 0.45 * got[0]
