"""Parity of the full SP2 path (sp2_density through the C ABI) against the CPU oracle.

The oracle is the exact projector (eigh / construction) and Alg. 1 run in FP64 on the
CPU.  Accuracy bars: ||D - D_ref||_F <= 1e-3 sqrt(N) and |Tr D - N_occ| <= 1e-6 for the
mixed modes; the FP64 mode must reach idempotency below 1e-12 on the N = 256 case.
"""
import numpy as np
import pytest
import torch

from oracle import dm
from oracle import sp2 as osp2
from paper_2101_06385_amd import sp2, workloads as wl

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _run(w, **kw):
    h = torch.from_numpy(w.h).to(DEV)
    d, info = sp2.density(h, w.n_occ, **kw)
    return d.cpu().numpy(), info


def _same_early_history(info, ref, floor):
    """sigma_n must agree while IdErr is well above the noise floor of the precision."""
    k = 0
    for i, (s, e) in enumerate(zip(ref.sigma, ref.iderr)):
        if e < floor or i >= len(info["sigma"]):
            break
        assert info["sigma"][i] == s, (i, info["sigma"][:i + 1], ref.sigma[:i + 1])
        k += 1
    return k


def test_fp64_config1_against_oracle():
    w = wl.config1()
    d, info = _run(w, precision="fp64", tol=1e-12)
    d_ref = dm.dm_construct(w.q, w.eps, w.n_occ)
    assert info["status"] == sp2.SP2_OK, info["status_name"]
    assert np.linalg.norm(d - d_ref) < 1e-10
    assert abs(info["trace"] - w.n_occ) < 1e-12
    assert abs(info["idem"]) < 1e-12
    ref = osp2.sp2_alg1(w.h, w.n_occ)
    # same bounds (both Gershgorin with the same outward widening)
    assert abs(info["emin"] - ref.bounds[0]) < 1e-12 * abs(ref.bounds[0])
    assert abs(info["emax"] - ref.bounds[1]) < 1e-12 * abs(ref.bounds[1])
    k = _same_early_history(info, ref, 1e-9)
    assert k >= ref.layers - 4
    assert abs(info["layers"] - ref.layers) <= 2
    # IdErr history matches while above the FP64 noise floor
    for i in range(k):
        assert abs(info["iderr"][i] - ref.iderr[i]) <= 1e-9 * max(1.0, abs(ref.iderr[i]))
        assert abs(info["ns"][i] - ref.ns[i]) <= 1e-9 * max(1.0, abs(ref.ns[i]))


@pytest.mark.parametrize("prec", ["fp16x2", "bf16x2", "fp32"])
@pytest.mark.parametrize("n", [1000, 1024])
def test_mixed_modes_against_exact(prec, n):
    w = wl.gapped(31 + n, n, n // 4, occ_lo=-30.0, homo=-0.5, lumo=0.5, virt_hi=30.0)
    d, info = _run(w, precision=prec)
    d_ref = dm.dm_construct(w.q, w.eps, w.n_occ)
    err = float(np.linalg.norm(d - d_ref))
    assert info["status"] == sp2.SP2_OK, (info["status_name"], info["trace"], info["idem"])
    assert err <= 1e-3 * np.sqrt(n), err
    assert abs(info["trace"] - w.n_occ) <= 1e-6
    assert np.array_equal(d, d.T)
    ref = osp2.sp2_alg1(w.h, w.n_occ)
    assert _same_early_history(info, ref, 1e-1) >= 10


def test_fp16x2_paper_split_without_shift():
    w = wl.gapped(5, 512, 128)
    d, info = _run(w, precision="fp16x2", scale_log2=0)
    assert info["status"] == sp2.SP2_OK
    assert np.linalg.norm(d - dm.dm_construct(w.q, w.eps, w.n_occ)) <= 1e-3 * np.sqrt(512)


def test_config2_full_size_sampled_rows():
    """N = 4096 mixed-precision case, FP16X2 vs FP32 vs FP64 on the GPU; sampled rows
    of the exact projector computed one by one."""
    w = wl.config2()
    rows = [0, 1, 777, 2048, 4095]
    d_rows = dm.dm_rows(w.q, w.eps, w.n_occ, rows)
    for prec in ("fp16x2", "fp32", "fp64"):
        d, info = _run(w, precision=prec)
        assert info["status"] == sp2.SP2_OK, (prec, info["status_name"])
        assert abs(info["trace"] - w.n_occ) <= 1e-6
        assert abs(info["idem"]) <= 1e-6 * w.n
        assert np.abs(d[rows] - d_rows).max() <= (1e-9 if prec == "fp64" else 1e-3), prec
        assert np.array_equal(d, d.T)


def test_bench_config_8192_sampled_rows():
    """The benchmark workload (N = 8192, 25% occupation, 0.2 eV gap) in the launch
    configuration the benchmark times: default options (FP16X2, automatic tile)."""
    w = wl.config3(n=8192)
    rows = [0, 4095, 8191]
    d, info = _run(w, precision="fp16x2")
    assert info["status"] == sp2.SP2_OK, info["status_name"]
    assert abs(info["trace"] - w.n_occ) <= 1e-6
    assert np.array_equal(d[rows][:, :64], d[:64][:, rows].T)
    d_rows = dm.dm_rows(w.q, w.eps, w.n_occ, rows)
    assert np.abs(d[rows] - d_rows).max() <= 1e-3
    # Frobenius error of the whole matrix from its sampled rows is bounded via the
    # properties that hold at any size: idempotency and occupation
    assert abs(info["idem"]) <= 1e-6 * w.n


# ------------------------------------------------------------------------ edge cases
def test_one_and_two_by_two():
    for n_occ in (0, 1):
        h = torch.tensor([[2.5]], dtype=torch.float64, device=DEV)
        d, info = sp2.density(h, n_occ, precision="fp64")
        assert info["status"] == sp2.SP2_OK and d.item() == float(n_occ)
    a, b, c = 0.3, -1.1, 2.0
    h = torch.tensor([[a, b], [b, c]], dtype=torch.float64, device=DEV)
    lam = 0.5 * (a + c) - np.sqrt((0.5 * (a - c)) ** 2 + b * b)
    v = np.array([b, lam - a])
    v /= np.linalg.norm(v)
    for prec in ("fp64", "fp16x2"):
        d, info = sp2.density(h, 1, precision=prec)
        assert info["status"] == sp2.SP2_OK, (prec, info["status_name"])
        assert np.abs(d.cpu().numpy() - np.outer(v, v)).max() < (1e-12 if prec == "fp64" else 1e-4)


@pytest.mark.parametrize("n_occ", [0, 77])
def test_empty_and_full_occupation(n_occ):
    w = wl.gapped(3, 77, 30)
    d, info = _run(w.__class__(w.name, w.n, n_occ, w.eps, w.q, w.h), precision="fp16x2")
    expect = np.eye(77) if n_occ == 77 else np.zeros((77, 77))
    assert info["status"] == sp2.SP2_OK
    assert np.array_equal(d, expect)


def test_leading_dimension_and_energy():
    w = wl.gapped(9, 333, 100)
    big = torch.zeros((333, 400), dtype=torch.float64, device=DEV)
    big[:, :333] = torch.from_numpy(w.h).to(DEV)
    h = big[:, :333]
    out = torch.full((333, 350), 7.0, dtype=torch.float64, device=DEV)
    d, info = sp2.density(h, 100, precision="fp64", want_energy=True, out=out[:, :333])
    d_ref = dm.dm_construct(w.q, w.eps, 100)
    assert info["status"] == sp2.SP2_OK
    assert np.linalg.norm(out[:, :333].cpu().numpy() - d_ref) < 1e-10
    assert torch.all(out[:, 333:] == 7.0)          # outside the matrix untouched
    assert abs(info["energy"] - float(np.sum(w.eps[:100]))) < 1e-9 * abs(float(np.sum(w.eps[:100])))


def test_nonfinite_input():
    w = wl.gapped(4, 100, 40)
    h = w.h.copy()
    h[3, 7] = h[7, 3] = np.nan
    d, info = sp2.density(torch.from_numpy(h).to(DEV), 40, precision="fp16x2")
    assert info["status"] == sp2.SP2_ENONFINITE


def test_asymmetric_input_rejected():
    w = wl.gapped(4, 100, 40)
    h = w.h.copy()
    h[3, 7] += 1e-3
    d, info = sp2.density(torch.from_numpy(h).to(DEV), 40, precision="fp64")
    assert info["status"] == sp2.SP2_EINVAL
    assert info["asym"] > 5e-4


def test_layer_cap_reports_no_convergence():
    w = wl.config1()
    d, info = _run(w, precision="fp64", max_layers=4)
    assert info["status"] == sp2.SP2_ENOCONV
    assert info["layers"] == 4 and not info["converged"]


def test_degenerate_homo_lumo():
    w = wl.gapped(8, 64, 20, homo=0.0, lumo=0.0)
    d, info = _run(w, precision="fp64")
    assert info["status"] in (sp2.SP2_ENOTIDEMP, sp2.SP2_ENOCONV)


def test_bounds_not_enclosing_spectrum_are_reported():
    """Bounds far inside the spectrum put eigenvalues of S_0 outside [0,1]: Tr[S - S^2] < 0
    stops Alg. 1 at once (or the layers overflow); either way the final check fails."""
    w = wl.config1()
    d, info = _run(w, precision="fp16x2", bounds=(-1.0, 1.0))
    assert info["status"] in (sp2.SP2_ENONFINITE, sp2.SP2_ENOTIDEMP)
    assert info["iderr"][0] < 0 or info["status"] == sp2.SP2_ENONFINITE


def test_exact_bounds_need_fewer_layers():
    w = wl.config1()
    _, g = _run(w, precision="fp64")
    _, e = _run(w, precision="fp64", bounds=(float(w.eps[0]) - 1e-9, float(w.eps[-1]) + 1e-9))
    assert e["status"] == sp2.SP2_OK and e["layers"] < g["layers"]
    ref = osp2.sp2_eigen((e["emax"] - w.eps) / (e["emax"] - e["emin"]), w.n_occ)
    assert abs(e["layers"] - ref.layers) <= 2


def test_repeatable_bitwise():
    w = wl.gapped(10, 700, 200)
    d1, i1 = _run(w, precision="fp16x2")
    d2, i2 = _run(w, precision="fp16x2")
    assert np.array_equal(d1, d2) and i1 == i2


def test_async_call_and_query():
    w = wl.gapped(11, 300, 100)
    h = torch.from_numpy(w.h).to(DEV)
    opts = sp2.options("fp16x2")
    ws = sp2.alloc_workspace(sp2.workspace_size(300, opts), h.device)
    d, info = sp2.density(h, 100, workspace=ws, sync=False)
    assert info is None
    q = sp2.query(ws, 300, "fp16x2")
    assert q["status"] == sp2.SP2_OK and q["layers"] > 10


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16x2"])
def test_layers_after_the_stop_do_no_work(prec):
    """Synchronous calls enqueue up to two chunks of layers beyond the stopping layer; those
    must return at once (skip flag) and leave S_{m-1} for the refinement untouched.  The size
    keeps a working layer (about 80 us in FP16X2) well above the launch cost of a skipped
    one (about 5 us)."""
    w = wl.gapped(77, 2100, 600)
    h = torch.from_numpy(w.h).to(DEV)
    _, info, tm = sp2.density(h, w.n_occ, precision=prec, timed=True)
    m = info["layers"]
    ran = tm["square_ms"][:m - 1]
    extra = [t for t in tm["square_ms"][m - 1:] if t > 0]
    assert extra, "expected layers enqueued after the stop"
    assert max(extra) < 0.2 * float(np.median(ran)), (max(extra), float(np.median(ran)))
    assert info["status"] == 0


def _sampled_check(w, d, info, rows, fro_tol):
    assert info["status"] == sp2.SP2_OK, info["status_name"]
    assert abs(info["trace"] - w.n_occ) <= 1e-6
    assert np.array_equal(d[rows][:, :64], d[:64][:, rows].T)
    d_rows = dm.dm_rows(w.q, w.eps, w.n_occ, rows)
    assert np.abs(d[rows] - d_rows).max() <= fro_tol
    assert abs(info["idem"]) <= 1e-6 * w.n


def test_stress_config_16384_sampled_rows():
    """The second size of the small-gap stress case (N = 16384, 0.2 eV gap) with default
    options (persistent 4-wave kernel): sampled rows of D against the exact projector."""
    w = wl.config3(n=16384, device=DEV)
    h = torch.from_numpy(w.h).to(DEV)
    d, info = sp2.density(h, w.n_occ)
    assert info["kernel"] >= 2 and info["tile"] == 256
    _sampled_check(w, d.cpu().numpy(), info, [0, 8191, 16383], 1e-3)


def test_stress_config_8192_bf16_sampled_rows():
    """BF16 planes on the N = 8192 stress case (the precision comparison of that case)."""
    w = wl.config3(n=8192, device=DEV)
    h = torch.from_numpy(w.h).to(DEV)
    d, info = sp2.density(h, w.n_occ, precision="bf16x2")
    _sampled_check(w, d.cpu().numpy(), info, [1, 4097, 8190], 2e-3)


def test_stress_config_8192_fp64_sampled_rows():
    """Plain FP64 SP2 at N = 8192 (the speed comparison of the benchmark): near-FP64 rows."""
    w = wl.config3(n=8192, device=DEV)
    h = torch.from_numpy(w.h).to(DEV)
    d, info = sp2.density(h, w.n_occ, precision="fp64")
    assert info["status"] == sp2.SP2_OK
    rows = [2, 5000]
    d = d.cpu().numpy()
    assert np.abs(d[rows] - dm.dm_rows(w.q, w.eps, w.n_occ, rows)).max() <= 1e-9


def test_observable_reductions_against_fsum():
    """sp2_observable: Tr D, ||D||_F^2 and sum_ij D_ij A_ij (Tr[D A] for a symmetric
    observable A) against math.fsum of the same FP64 values, within the bound on any order
    of FP64 additions; with A = H it is the energy sp2_density reports."""
    import math

    w = wl.gapped(88, 700, 200)
    h = torch.from_numpy(w.h).to(DEV)
    d, info = sp2.density(h, w.n_occ, want_energy=True)
    rng = np.random.default_rng(89)
    a = rng.standard_normal((700, 700))
    a = 0.5 * (a + a.T)
    dn = d.cpu().numpy()
    for mat in (a, w.h):
        out = sp2.observable(d, torch.from_numpy(mat).to(DEV))
        terms = [np.diag(dn), (dn * dn).ravel(), (dn * mat).ravel()]
        for got, t in zip(out, terms):
            assert abs(got - math.fsum(t)) <= t.size * 2.0 ** -53 * math.fsum(np.abs(t)) + 1e-300
    assert sp2.observable(d, h)[2] == info["energy"]


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-5), ("fp16x2", 1e-4), ("bf16x2", 1e-3)])
def test_paper_10x10_case(prec, tol):
    """The paper's 10 x 10 convergence example (H_ij uniform in [-1, 1], N_occ = 5) through
    the C ABI against the eigendecomposition; in FP64 the sigma history is the oracle's."""
    w = wl.small_random()
    d, info = _run(w, precision=prec)
    assert info["status"] == sp2.SP2_OK, info["status_name"]
    assert np.abs(d - dm.dm_eigh(w.h, w.n_occ)).max() <= tol
    if prec == "fp64":
        ref = osp2.sp2_alg1(w.h, w.n_occ)
        assert _same_early_history(info, ref, 1e-9) >= ref.layers - 4
