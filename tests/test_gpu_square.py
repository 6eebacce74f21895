"""Parity of one squaring layer on the GPU (the hot kernel) against the CPU oracle.

Split modes: compared with the oracle's Alg. 2 product of the SAME half-precision planes
(exact products, FP64 accumulation); the only difference allowed is FP32 accumulation,
bounded by  |dY| <= 2 K u (|X0||X0| + 2 |X0||X1|) 2^-2s |alpha|  plus one rounding of the
epilogue, with u = 2^-24 and K the product length.  FP32/FP64 modes: the same bound with
|X||X|.  Every result must be bitwise symmetric, and the FP64 tile sums must equal the
trace and squared Frobenius norm of the returned matrix.
"""
import math

import numpy as np
import pytest
import torch

from oracle import sp2 as osp2
from paper_2101_06385_amd import sp2, workloads as wl

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
U32 = 2.0 ** -24
COEFS = [(1.0, 0.0, 0.0), (-1.0, 2.0, 0.0), (0.75, -0.25, 0.125)]


def _state(n, seed):
    w = wl.gapped(seed, n, max(1, n // 3))
    return osp2.rescale(w.h, *osp2.gershgorin(w.h))


def _check_sums(y, sums):
    """The device's FP64 tile sums of Tr Y and ||Y||_F^2 against math.fsum (the exactly
    rounded sums of the same stored values; squares of FP32 values are exact in FP64):
    any order of FP64 additions of m terms is within (m - 1) 2^-53 sum |terms|."""
    y = np.asarray(y, dtype=np.float64)
    d = np.diag(y)
    sq = (y * y).ravel()
    tr = math.fsum(d)
    fr = math.fsum(sq)
    assert abs(sums[0] - tr) <= d.size * 2.0 ** -53 * math.fsum(np.abs(d)) + 1e-300
    assert abs(sums[1] - fr) <= sq.size * 2.0 ** -53 * fr + 1e-300


@pytest.mark.parametrize("prec,tile,n", [
    ("fp16x2", 64, 200), ("fp16x2", 128, 300), ("fp16x2", 256, 520), ("fp16x2", 256, 1024),
    ("bf16x2", 64, 130), ("bf16x2", 128, 300), ("bf16x2", 256, 600), ("fp16x2", 128, 1000),
])
def test_split_square_vs_exact_products(prec, tile, n):
    fmt = "fp16" if prec == "fp16x2" else "bf16"
    s = 12 if fmt == "fp16" else 0
    x = _state(n, 100 + n).astype(np.float32)
    x0, x1 = osp2.split_planes(x, fmt, s)
    a0, a1 = np.abs(x0.astype(np.float64)), np.abs(x1.astype(np.float64))
    mag = (a0 @ a0 + 2.0 * (a0 @ a1)) * 2.0 ** (-2 * s)
    x2 = osp2.mixed_square(x, fmt, s)
    xt = torch.from_numpy(x).to(DEV)
    for alpha, beta, gamma in COEFS:
        y, sums = sp2.square(xt, alpha, beta, gamma, precision=prec, tile=tile)
        y = y.cpu().numpy().astype(np.float64)
        assert np.array_equal(y, y.T), "not bitwise symmetric"
        ref = alpha * x2 + beta * x.astype(np.float64) + gamma * np.eye(n)
        bound = 2.0 * n * U32 * mag * abs(alpha) + 2.0 * U32 * (np.abs(alpha * x2) + abs(beta) * np.abs(x) + abs(gamma))
        err = np.abs(y - ref)
        assert np.all(err <= bound + 1e-30), (prec, tile, n, alpha, float((err / (bound + 1e-30)).max()))
        _check_sums(y, sums)


@pytest.mark.parametrize("prec,tile,n", [("fp64", 64, 100), ("fp64", 128, 260), ("fp32", 64, 150),
                                         ("fp32", 128, 384)])
def test_plain_square_vs_fp64(prec, tile, n):
    x = _state(n, 200 + n)
    dt = np.float64 if prec == "fp64" else np.float32
    u = 2.0 ** -53 if prec == "fp64" else U32
    x = x.astype(dt)
    xd = x.astype(np.float64)
    x2 = xd @ xd
    mag = np.abs(xd) @ np.abs(xd)
    xt = torch.from_numpy(x).to(DEV)
    for alpha, beta, gamma in COEFS:
        y, sums = sp2.square(xt, alpha, beta, gamma, precision=prec, tile=tile)
        y = y.cpu().numpy().astype(np.float64)
        assert np.array_equal(y, y.T)
        ref = alpha * x2 + beta * xd + gamma * np.eye(n)
        bound = 2.0 * n * u * mag * abs(alpha) + 2.0 * u * (np.abs(alpha * x2) + abs(beta) * np.abs(xd) + abs(gamma))
        err = np.abs(y - ref)
        assert np.all(err <= bound + 1e-300), (prec, tile, n, float((err / (bound + 1e-300)).max()))
        _check_sums(y, sums)


@pytest.mark.parametrize("prec,tile,kernel,n", [
    ("fp16x2", 256, 2, 6100), ("fp16x2", 256, 3, 6100), ("fp16x2", 256, 4, 6100), ("fp16x2", 256, 5, 6100),
    ("fp16x2", 128, 2, 4100), ("fp16x2", 128, 3, 4100), ("fp16x2", 128, 4, 4100), ("fp16x2", 128, 5, 4100),
    ("fp16x2", 256, 6, 6100), ("fp16x2", 256, 7, 6100), ("fp16x2", 128, 6, 4100), ("fp16x2", 128, 7, 4100),
    ("bf16x2", 256, 3, 6100), ("bf16x2", 128, 3, 4100), ("bf16x2", 256, 7, 6100), ("fp16x2", 256, 1, 6100),
    ("fp16x2", 128, 1, 4100), ("bf16x2", 128, 1, 4100), ("fp16x2", 256, 8, 6100), ("fp16x2", 128, 8, 4100),
    ("fp16x2", 256, 7, 8000), ("bf16x2", 256, 5, 8000),
])
def test_persistent_schedules_sampled_rows(prec, tile, kernel, n):
    """Persistent schedules, every kernel variant (only used once there are at least as
    many tiles as workgroups, hence the large n; 300 and 561 tiles leave a split tail in
    5 and 2 chunks per tile, summed in one level; n = 8000 pads to 528 tiles of 256, whose
    16 leftover tiles are cut into 16 chunks and summed in two levels of 4): sampled rows
    against the oracle's exact products."""
    fmt = "fp16" if prec == "fp16x2" else "bf16"
    s = 12 if fmt == "fp16" else 0
    rng = np.random.default_rng(n + kernel)
    a = rng.standard_normal((n, n)).astype(np.float32) / np.float32(np.sqrt(n))
    x = (a + a.T) * np.float32(0.5)
    rows = [0, 1, 255, 256, 1000, n // 2, n - 1]
    x0, x1 = osp2.split_planes(x, fmt, s)
    a0, a1 = np.abs(x0.astype(np.float64)), np.abs(x1.astype(np.float64))
    mag = (a0[rows] @ a0 + a0[rows] @ a1 + a1[rows] @ a0) * 2.0 ** (-2 * s)
    ref = osp2.mixed_square_rows(x, rows, fmt, s)
    for alpha, beta, gamma in COEFS[:2]:
        y, sums = sp2.square(torch.from_numpy(x).to(DEV), alpha, beta, gamma, precision=prec, tile=tile,
                             kernel=kernel)
        assert torch.equal(y, y.T)
        yr = y[rows].cpu().numpy().astype(np.float64)
        want = alpha * ref + beta * x[rows].astype(np.float64) + gamma * np.eye(n)[rows]
        bound = 2.0 * n * U32 * mag + 2.0 * U32 * (np.abs(alpha * ref) + abs(beta) * np.abs(x[rows]))
        err = np.abs(yr - want)
        assert np.all(err <= bound + 1e-30), float((err / (bound + 1e-30)).max())
        tr = float(torch.trace(y.double()))
        fr = float((y.double() ** 2).sum())
        assert abs(sums[0] - tr) <= 1e-10 * max(1.0, abs(tr)) and abs(sums[1] - fr) <= 1e-10 * fr


@pytest.mark.parametrize("prec,tile,kernel,n", [
    ("fp16x2", 128, 5, 2048), ("fp16x2", 128, 4, 2048), ("fp16x2", 128, 5, 3000), ("bf16x2", 128, 5, 3000),
    ("fp16x2", 256, 5, 4096), ("fp16x2", 256, 4, 3000), ("fp16x2", 128, 7, 1500),
    ("fp16x2", 256, 7, 3000), ("bf16x2", 256, 7, 4096), ("fp16x2", 256, 6, 3000), ("fp16x2", 128, 6, 2048),
])
def test_stream_k_schedules_sampled_rows(prec, tile, kernel, n):
    """Fewer tiles than workgroups: the persistent kernel splits the K-slices of all tiles
    evenly over the workgroups (stream-K), and the tiles shared by several ranges are summed
    by their last contributor.  Sizes with several tiles per range, several ranges per tile
    and ragged edges; sampled rows against the oracle's exact products of the same planes."""
    fmt = "fp16" if prec == "fp16x2" else "bf16"
    s = 12 if fmt == "fp16" else 0
    rng = np.random.default_rng(n + 10 * kernel + tile)
    a = rng.standard_normal((n, n)).astype(np.float32) / np.float32(np.sqrt(n))
    x = (a + a.T) * np.float32(0.5)
    rows = sorted({0, 1, 127, 128, 255, 256, n // 3, n // 2, n - 2, n - 1})
    x0, x1 = osp2.split_planes(x, fmt, s)
    a0, a1 = np.abs(x0.astype(np.float64)), np.abs(x1.astype(np.float64))
    mag = (a0[rows] @ a0 + a0[rows] @ a1 + a1[rows] @ a0) * 2.0 ** (-2 * s)
    ref = osp2.mixed_square_rows(x, rows, fmt, s)
    xt = torch.from_numpy(x).to(DEV)
    outs = []
    for alpha, beta, gamma in COEFS:
        y, sums = sp2.square(xt, alpha, beta, gamma, precision=prec, tile=tile, kernel=kernel)
        assert torch.equal(y, y.T)
        yr = y[rows].cpu().numpy().astype(np.float64)
        want = alpha * ref + beta * x[rows].astype(np.float64) + gamma * np.eye(n)[rows]
        bound = 2.0 * n * U32 * mag * abs(alpha) + 2.0 * U32 * (np.abs(alpha * ref) + abs(beta) * np.abs(x[rows])
                                                               + abs(gamma))
        err = np.abs(yr - want)
        assert np.all(err <= bound + 1e-30), float((err / (bound + 1e-30)).max())
        tr = float(torch.trace(y.double()))
        fr = float((y.double() ** 2).sum())
        assert abs(sums[0] - tr) <= 1e-10 * max(1.0, abs(tr)) and abs(sums[1] - fr) <= 1e-10 * fr
        outs.append(y)
    # the fixed summation order makes the result reproducible bit for bit
    y2, _ = sp2.square(xt, *COEFS[-1], precision=prec, tile=tile, kernel=kernel)
    assert torch.equal(outs[-1], y2)


@pytest.mark.parametrize("n,tile,kernel", [(2048, 128, 5), (3000, 256, 5)])
def test_stream_k_schedule_in_the_density_path(n, tile, kernel):
    """The whole path with a stream-K squaring schedule reports it and reaches the exact
    projector (accuracy bar of the mixed modes)."""
    from oracle import dm

    w = wl.gapped(41 + n, n, n // 4, occ_lo=-30.0, homo=-0.5, lumo=0.5, virt_hi=30.0)
    d, info = sp2.density(torch.from_numpy(w.h).to(DEV), w.n_occ, tile=tile, kernel=kernel)
    assert info["kernel"] == kernel and info["tile"] == tile
    assert info["status"] == sp2.SP2_OK, info["status_name"]
    d = d.cpu().numpy()
    assert np.array_equal(d, d.T)
    assert np.linalg.norm(d - dm.dm_construct(w.q, w.eps, w.n_occ)) <= 1e-3 * np.sqrt(n)
    assert abs(info["trace"] - w.n_occ) <= 1e-6


def test_persistent_schedule_deterministic():
    n = 6100
    rng = np.random.default_rng(1)
    a = rng.standard_normal((n, n)).astype(np.float32) / np.float32(np.sqrt(n))
    x = torch.from_numpy((a + a.T) * np.float32(0.5)).to(DEV)
    y1, s1 = sp2.square(x, precision="fp16x2", tile=256, kernel=2)
    y2, s2 = sp2.square(x, precision="fp16x2", tile=256, kernel=2)
    assert torch.equal(y1, y2) and s1 == s2


def test_split_square_paper_mode_without_shift():
    """scale_log2 = 0 is the paper's split exactly (Eqs. Split1/Split2)."""
    n = 256
    x = _state(n, 7).astype(np.float32)
    y, _ = sp2.square(torch.from_numpy(x).to(DEV), precision="fp16x2", tile=128, scale_log2=0)
    x0, x1 = osp2.split_planes(x, "fp16", 0)
    a0, a1 = np.abs(x0.astype(np.float64)), np.abs(x1.astype(np.float64))
    bound = 2.0 * n * U32 * (a0 @ a0 + 2 * a0 @ a1) + 2 * U32 * np.abs(osp2.mixed_square(x, "fp16", 0))
    assert np.all(np.abs(y.cpu().numpy() - osp2.mixed_square(x, "fp16", 0)) <= bound)


def test_square_is_deterministic():
    x = torch.from_numpy(_state(700, 3).astype(np.float32)).to(DEV)
    y1, s1 = sp2.square(x, precision="fp16x2", tile=256)
    y2, s2 = sp2.square(x, precision="fp16x2", tile=256)
    assert torch.equal(y1, y2) and s1 == s2


@pytest.mark.parametrize("kernel", [0, 1, 2, 3, 4, 5])
def test_fp64_kernels_vs_exact(kernel):
    """The FP64 layer kernels (register-staged, direct-to-LDS variants) on a
    ragged size that spans several 128 tiles: each within the FP64 accumulation bound of
    the exact product, all bitwise symmetric."""
    n = 900
    x = _state(n, 300)
    x2 = x @ x
    mag = np.abs(x) @ np.abs(x)
    u = 2.0 ** -53
    for alpha, beta, gamma in COEFS:
        y, sums = sp2.square(torch.from_numpy(x).to(DEV), alpha, beta, gamma, precision="fp64", tile=128,
                             kernel=kernel)
        y = y.cpu().numpy()
        assert np.array_equal(y, y.T)
        ref = alpha * x2 + beta * x + gamma * np.eye(n)
        bound = 2.0 * n * u * mag * abs(alpha) + 2.0 * u * (np.abs(alpha * x2) + abs(beta) * np.abs(x) + abs(gamma))
        assert np.all(np.abs(y - ref) <= bound + 1e-300), kernel
        _check_sums(y, sums)


@pytest.mark.parametrize("kernel", [5, 4])
def test_fp64_persistent_schedule_sampled_rows(kernel):
    """The persistent FP64 layer (whole rounds, split-K tail; 2080 tiles of 128 at n = 8150
    leave a tail on 256 CUs) against exact FP64 products of sampled rows, twice in a row
    (the arrival counters carry over between launches)."""
    n = 8150
    rng = np.random.default_rng(11)
    a = rng.standard_normal((n, n)) / np.sqrt(n)
    x = (a + a.T) * 0.5
    rows = [0, 127, 128, 4000, n - 1]
    ref = x[rows] @ x
    mag = np.abs(x[rows]) @ np.abs(x)
    xt = torch.from_numpy(x).to(DEV)
    ws = sp2.alloc_workspace(sp2.lib().sp2_square_workspace_size(n, sp2.FP64, 128, kernel), xt.device)
    for _ in range(2):
        y, sums = sp2.square(xt, 1.0, 0.0, 0.0, precision="fp64", tile=128, kernel=kernel, workspace=ws)
        yr = y[rows].cpu().numpy()
        assert np.all(np.abs(yr - ref) <= 2.0 * n * 2.0 ** -53 * mag + 1e-300)
        assert torch.equal(y, y.T)
        tr = float(torch.trace(y))
        assert abs(sums[0] - tr) <= 1e-10 * abs(tr)
