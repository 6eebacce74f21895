"""Parity of the accelerated Deep-NN SP2 layers (Sec. Accelerated Deep-NN SP2) on the GPU
against the CPU oracle's accelerated run and the exact projector.

The accelerated choices depend only on the spectral bounds and the caller's HOMO/LUMO
interval, not on rounding, so their sign sequence and real weights must agree with the
oracle's exactly (weights to FP64 rounding); the layers of Alg. 1 that follow are
compared as in the plain SP2 tests.
"""
import numpy as np
import pytest
import torch

from oracle import dm
from oracle import sp2 as osp2
from paper_2101_06385_amd import sp2, workloads as wl

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _run(h, n_occ, **kw):
    d, info = sp2.density(torch.from_numpy(h).to(DEV), n_occ, **kw)
    return d.cpu().numpy(), info


def _check_accelerated_history(info, ref):
    k = ref.accelerated
    assert k > 0 and info["accelerated"] == k, (info["accelerated"], k)
    assert info["gap_violation"] == 0 and ref.gap_violation == 0
    assert info["sigma"][:k] == ref.sigma[:k]
    got = np.array(info["sigma_c"][:k])
    assert np.allclose(got, ref.sigma_c[:k], rtol=1e-12, atol=0.0), (got, ref.sigma_c[:k])


@pytest.mark.parametrize("case", [(51, 300, 75, -1.0, 1.0), (52, 257, 200, 6.0, 6.2), (53, 320, 40, -15.0, -14.9)])
def test_fp64_accelerated_against_oracle(case):
    seed, n, n_occ, homo, lumo = case
    w = wl.gapped(seed, n, n_occ, occ_lo=-20.0, homo=homo, lumo=lumo, virt_hi=20.0)
    d, info = _run(w.h, w.n_occ, precision="fp64", tol=1e-12, gap=(w.homo, w.lumo))
    ref = osp2.sp2_accelerated(w.h, w.n_occ, w.homo, w.lumo)
    std = osp2.sp2_alg1(w.h, w.n_occ)
    assert info["status"] == sp2.SP2_OK, info["status_name"]
    assert np.linalg.norm(d - dm.dm_construct(w.q, w.eps, w.n_occ)) < 1e-10
    assert abs(info["idem"]) < 1e-12
    _check_accelerated_history(info, ref)
    # the accelerated layers run with their FP64 coefficients: the traces of every layer
    # through the first ordinary one follow the oracle's to FP64 rounding (about 1e-15
    # between two FP64 evaluations; FP32-rounded coefficients would show about 1e-8)
    for i in range(ref.accelerated + 1):
        assert abs(info["ns"][i] - ref.ns[i]) <= 1e-12 * max(1.0, abs(ref.ns[i])), (i, info["ns"][i], ref.ns[i])
        assert abs(info["nx"][i] - ref.nx[i]) <= 1e-12 * max(1.0, abs(ref.nx[i])), (i, info["nx"][i], ref.nx[i])
    assert np.abs(d - ref.d).max() <= 1e-12
    # Alg. 1 layers after the accelerated ones: same signs while IdErr is above the FP64 floor
    for i in range(ref.accelerated, ref.layers):
        if ref.iderr[i] < 1e-9:
            break
        assert info["sigma"][i] == ref.sigma[i], i
    assert abs(info["layers"] - ref.layers) <= 2
    assert info["layers"] < std.layers


@pytest.mark.parametrize("prec", ["fp16x2", "bf16x2", "fp32"])
def test_mixed_accelerated_against_exact(prec):
    n = 1000
    w = wl.gapped(61, n, n // 4, occ_lo=-30.0, homo=-0.5, lumo=0.5, virt_hi=30.0)
    d, info = _run(w.h, w.n_occ, precision=prec, gap=(w.homo, w.lumo))
    _, plain = _run(w.h, w.n_occ, precision=prec)
    ref = osp2.sp2_accelerated(w.h, w.n_occ, w.homo, w.lumo)
    assert info["status"] == sp2.SP2_OK, (info["status_name"], info["trace"], info["idem"])
    assert np.linalg.norm(d - dm.dm_construct(w.q, w.eps, w.n_occ)) <= 1e-3 * np.sqrt(n)
    assert abs(info["trace"] - w.n_occ) <= 1e-6
    assert np.array_equal(d, d.T)
    _check_accelerated_history(info, ref)
    assert info["layers"] < plain["layers"]


def test_stress_config_8192_accelerated_sampled_rows():
    """The N = 8192 small-gap stress case with its HOMO/LUMO values given: sampled rows of
    D against the exact projector, and far fewer layers than plain Alg. 1 (56 -> about 31
    in the FP64 eigenvalue recursion)."""
    w = wl.config3(n=8192, device=DEV)
    h = torch.from_numpy(w.h).to(DEV)
    d, info = sp2.density(h, w.n_occ, gap=(w.homo, w.lumo))
    _, plain = sp2.density(h, w.n_occ)
    assert info["status"] == sp2.SP2_OK, info["status_name"]
    assert abs(info["trace"] - w.n_occ) <= 1e-6 and abs(info["idem"]) <= 1e-6 * w.n
    rows = [0, 3000, 8191]
    d = d.cpu().numpy()
    assert np.array_equal(d[rows][:, :64], d[:64][:, rows].T)
    assert np.abs(d[rows] - dm.dm_rows(w.q, w.eps, w.n_occ, rows)).max() <= 1e-3
    e1, en = info["emin"], info["emax"]
    lam0 = (en - w.eps) / (en - e1)
    l0, h0 = osp2.homo_lumo_rescaled(w.homo, w.lumo, e1, en)
    ref = osp2.sp2_eigen_accelerated(lam0, w.n_occ, l0, h0)
    _check_accelerated_history(info, ref)
    assert info["layers"] <= plain["layers"] - 15, (info["layers"], plain["layers"])


def test_gap_outside_the_bounds_runs_plain_alg1():
    """HOMO/LUMO values that do not rescale into [0, 1]: no accelerated layer, and the
    result is bit-identical to a call without them."""
    w = wl.gapped(71, 400, 100)
    d0, i0 = _run(w.h, w.n_occ)
    d1, i1 = _run(w.h, w.n_occ, gap=(-1e9, 1e9))
    assert i1["accelerated"] == 0 and i0["accelerated"] == 0
    assert i1["layers"] == i0["layers"] and np.array_equal(d0, d1)


def test_tiny_spectra_accelerated_fp64():
    """Tiny systems (n = 2..5) with exact bounds: IdErr is small while layers are still
    accelerated, the case the stopping rule's restriction is for.  D must be the exact
    projector and the history the oracle's."""
    rng = np.random.default_rng(81)
    for _ in range(24):
        n = int(rng.integers(2, 6))
        n_occ = int(rng.integers(1, n))
        gap = 10 ** rng.uniform(-5, -0.5)
        c = rng.uniform(0.01 + gap, 0.99 - gap)
        l, h = c - gap / 2, c + gap / 2
        un = np.sort(rng.uniform(0.0, l, n - n_occ))
        un[-1] = l
        oc = np.sort(rng.uniform(h, 1.0, n_occ))
        oc[0] = h
        lam = np.concatenate([oc[::-1], un[::-1]])       # S-space eigenvalues, occupied first
        eps = 1.0 - lam                                   # H = (1 - S) with bounds [0, 1]: ascending
        q = wl.haar_orthogonal(rng, n)
        hm = wl.symmetric_from_eigen(q, eps)
        homo, lumo = 1.0 - h, 1.0 - l
        d, info = _run(hm, n_occ, precision="fp64", bounds=(0.0, 1.0), gap=(homo, lumo))
        ref = osp2.sp2_accelerated(hm, n_occ, homo, lumo, bounds=(0.0, 1.0))
        assert np.abs(d - dm.dm_construct(q, eps, n_occ)).max() < 1e-9, (n, n_occ, l, h)
        assert info["accelerated"] == ref.accelerated and info["sigma"][:ref.accelerated] == ref.sigma[:ref.accelerated]


@pytest.mark.parametrize("prec", ["fp64", "fp16x2"])
def test_interval_inside_a_band_is_reported(prec):
    """An interval inside the occupied or the virtual band (not inside the gap) ends on an
    idempotent projector with the right trace but onto the wrong states; the per-layer
    interval check must report it (SP2_ENOTIDEMP, gap_violation > 0), at the layer the
    oracle's check names in FP64."""
    w = wl.gapped(91, 400, 100, occ_lo=-20.0, homo=-1.0, lumo=1.0, virt_hi=20.0)
    for homo, lumo in ((-10.0, -5.0), (5.0, 10.0)):
        d, info = _run(w.h, w.n_occ, precision=prec, gap=(homo, lumo))
        ref = osp2.sp2_accelerated(w.h, w.n_occ, homo, lumo)
        assert ref.gap_violation > 0
        assert info["status"] == sp2.SP2_ENOTIDEMP, info["status_name"]
        assert info["gap_violation"] > 0
        if prec == "fp64":
            assert info["gap_violation"] == ref.gap_violation


def test_stress_config_16384_accelerated_sampled_rows():
    """The second size of the stress case with its HOMO/LUMO values (persistent 4-wave
    kernel): sampled rows against the exact projector and the oracle's accelerated
    history on the eigenvalues."""
    w = wl.config3(n=16384, device=DEV)
    h = torch.from_numpy(w.h).to(DEV)
    d, info = sp2.density(h, w.n_occ, gap=(w.homo, w.lumo))
    assert info["status"] == sp2.SP2_OK and info["gap_violation"] == 0, info["status_name"]
    rows = [5, 9000, 16383]
    d = d.cpu().numpy()
    assert np.abs(d[rows] - dm.dm_rows(w.q, w.eps, w.n_occ, rows)).max() <= 1e-3
    assert np.array_equal(d[rows][:, :64], d[:64][:, rows].T)
    e1, en = info["emin"], info["emax"]
    lam0 = (en - w.eps) / (en - e1)
    l0, h0 = osp2.homo_lumo_rescaled(w.homo, w.lumo, e1, en)
    _check_accelerated_history(info, osp2.sp2_eigen_accelerated(lam0, w.n_occ, l0, h0))
