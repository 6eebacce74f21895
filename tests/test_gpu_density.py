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


def _check_first_sign(info, ref):
    """Refinement reading R5: the first composed step takes -sigma_{m-1} (+1 after sigma_0 = 0).
    The GPU's choice follows its own history, and equals the oracle's whenever the two
    histories agree through layer m - 1."""
    m = info["layers"]
    last = info["sigma"][m - 2] if m >= 2 else 0
    assert info["first_sign"] == (-last if last else 1)
    if m == ref.layers and info["sigma"][:m - 1] == ref.sigma[:m - 1]:
        assert info["first_sign"] == ref.first_sign


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
    _check_first_sign(info, ref)
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


def _full_error_check(w, d, info, bar_rel=1e-3):
    """The accuracy bar of the mixed modes on the whole matrix: ||D - D_ref||_F <= 1e-3 sqrt(N)
    with D_ref = Q_occ Q_occ^T from the construction (one FP64 product on the host), plus
    |Tr D - N_occ| <= 1e-6 and exact symmetry."""
    assert info["status"] == sp2.SP2_OK, info["status_name"]
    assert abs(info["trace"] - w.n_occ) <= 1e-6
    d_ref = dm.dm_construct(w.q, w.eps, w.n_occ)
    d_ref -= d
    err = float(np.linalg.norm(d_ref))
    print("%s: ||D - D_ref||_F = %.3e (bar %.3e)" % (w.name, err, bar_rel * np.sqrt(w.n)), flush=True)
    assert err <= bar_rel * np.sqrt(w.n), err
    return err


def test_bench_config_8192_full_matrix():
    """The benchmark workload (N = 8192, 25% occupation, 0.2 eV gap) in the launch
    configuration the benchmark times (default options: FP16X2, automatic schedule): the
    whole D against the exact projector."""
    w = wl.config3(n=8192, device=DEV)
    h = torch.from_numpy(w.h).to(DEV)
    d, info = sp2.density(h, w.n_occ, precision="fp16x2")
    d = d.cpu().numpy()
    assert np.array_equal(d, d.T)
    _full_error_check(w, d, info)


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


def test_stress_config_16384_full_matrix():
    """The second size of the small-gap stress case (N = 16384, 0.2 eV gap) with default
    options (persistent kernel): the whole D against the exact projector."""
    w = wl.config3(n=16384, device=DEV)
    h = torch.from_numpy(w.h).to(DEV)
    d, info = sp2.density(h, w.n_occ)
    assert info["kernel"] >= 2 and info["tile"] == 256
    d = d.cpu().numpy()
    _full_error_check(w, d, info)
    assert np.array_equal(d[:, :64], d[:64].T)


def test_stress_config_8192_bf16_full_matrix():
    """BF16 planes on the N = 8192 stress case (the precision comparison of that case): the
    whole D against the exact projector."""
    w = wl.config3(n=8192, device=DEV)
    h = torch.from_numpy(w.h).to(DEV)
    d, info = sp2.density(h, w.n_occ, precision="bf16x2")
    d = d.cpu().numpy()
    assert np.array_equal(d, d.T)
    _full_error_check(w, d, info)


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


# ------------------------------------------------------------------------ eps term and ties of Alg. 1
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_fp64_large_eps_alternates_like_the_oracle(seed):
    """Alg. 1 with eps far above N: from layer 2 on every sign is the opposite of the previous
    one, on the GPU as in the oracle, and D is the same projector (onto the eigenvalues of S_0
    beyond the repelling fixed point of the two-step map)."""
    w = wl.gapped(300 + seed, 90, 20 + 10 * seed)
    bounds = osp2.gershgorin(w.h)
    ref = osp2.sp2_alg1(w.h, w.n_occ, eps=1e9, bounds=bounds)
    d, info = _run(w, precision="fp64", eps=1e9, bounds=bounds)
    m = info["layers"]
    assert info["converged"]
    assert all(info["sigma"][i] == -info["sigma"][i - 1] for i in range(1, m)), info["sigma"][:m]
    assert info["sigma"][0] == ref.sigma[0]
    assert abs(m - ref.layers) <= 1
    _check_first_sign(info, ref)
    assert np.abs(d - ref.d).max() < 1e-9
    lam0 = (bounds[1] - w.eps) / (bounds[1] - bounds[0])
    thr = (np.sqrt(5.0) - 1.0) / 2.0 if ref.sigma[0] > 0 else (3.0 - np.sqrt(5.0)) / 2.0
    keep = lam0 > thr
    assert np.abs(d - w.q[:, keep] @ w.q[:, keep].T).max() < 1e-9


def test_fp64_moderate_eps_history_like_the_oracle():
    """A moderate eps changes some sign decisions near convergence; the GPU's signs equal the
    oracle's wherever IdErr is above the FP64 noise floor, and D is exact."""
    w = wl.gapped(310, 200, 60)
    bounds = osp2.gershgorin(w.h)
    for eps in (0.5, 3.0):
        ref = osp2.sp2_alg1(w.h, w.n_occ, eps=eps, bounds=bounds)
        plain = osp2.sp2_alg1(w.h, w.n_occ, bounds=bounds)
        d, info = _run(w, precision="fp64", eps=eps, bounds=bounds)
        assert info["status"] == sp2.SP2_OK, info["status_name"]
        assert _same_early_history(info, ref, 1e-9) >= ref.layers - 3
        assert abs(info["layers"] - ref.layers) <= 1
        _check_first_sign(info, ref)
        assert np.abs(d - dm.dm_construct(w.q, w.eps, w.n_occ)).max() < 1e-10
        if eps == 3.0:
            assert ref.sigma != plain.sigma   # the eps term is exercised


@pytest.mark.parametrize("lam,n_occ,tie_layer", [
    ([0.25, 0.75, 0.25, 0.75], 2, 1),
    ([1 / 16, 3 / 16, 9 / 16, 14 / 16, 15 / 16], 2, 2),
])
def test_fp64_exact_tie_like_the_oracle(lam, n_occ, tie_layer):
    """Sign(0) reading on dyadic spectra with exact traces: a tie at layer 1 (sigma_0 = 0) takes
    +1, a tie at layer 2 takes -sigma_1.  Diagonal H with bounds [0, 1] makes S_0 = diag(lam)
    exactly, so the GPU's measured traces are the oracle's exactly through the tie."""
    lam = np.array(lam)
    h = np.diag(1.0 - lam)
    ref = osp2.sp2_alg1(h, n_occ, bounds=(0.0, 1.0))
    d, info = sp2.density(torch.from_numpy(h).to(DEV), n_occ, precision="fp64", bounds=(0.0, 1.0), tol=1e-12)
    d = d.cpu().numpy()
    assert info["status"] == sp2.SP2_OK, info["status_name"]
    assert info["ns"][tie_layer - 1] == float(n_occ)
    want = 1 if tie_layer == 1 else -info["sigma"][tie_layer - 2]
    assert info["sigma"][tie_layer - 1] == want == ref.sigma[tie_layer - 1]
    assert info["sigma"][:tie_layer + 2] == ref.sigma[:tie_layer + 2]
    assert _same_early_history(info, ref, 1e-9) >= ref.layers - 3
    _check_first_sign(info, ref)
    expect = np.diag((lam > np.sort(lam)[-n_occ - 1]).astype(float))
    assert np.abs(d - expect).max() < 1e-12
