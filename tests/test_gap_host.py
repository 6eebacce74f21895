"""Host side of the HOMO/LUMO estimate in libsp2 (no GPU): sp2_estimate_gap against the
oracle's estimate on the same histories (FP64 eigenvalue runs, plain and accelerated),
and its argument errors."""
import ctypes

import numpy as np

from oracle import sp2 as osp2
from paper_2101_06385_amd import sp2


def _history(run):
    sc = getattr(run, "sigma_c", None) or [float(s) for s in run.sigma]
    return {"layers": run.layers, "sigma_c": list(sc), "iderr": list(run.iderr)}


def test_library_estimate_matches_oracle():
    rng = np.random.default_rng(53)
    compared = 0
    for t in range(120):
        n = int(rng.integers(20, 600))
        n_occ = int(rng.integers(1, n))
        homo = rng.uniform(-15.0, 15.0)
        gap = 10 ** rng.uniform(-2.0, 0.5)
        occ = np.sort(rng.uniform(-20.0, homo, n_occ))
        occ[-1] = homo
        vir = np.sort(rng.uniform(homo + gap, 25.0, n - n_occ))
        vir[0] = homo + gap
        eps = np.concatenate([occ, vir])
        e1, en = -30.0, 30.0
        lam0 = (en - eps) / (en - e1)
        runs = [osp2.sp2_eigen(lam0, n_occ)]
        if t % 2:
            runs.append(osp2.sp2_eigen_accelerated(lam0, n_occ, lam0[n_occ], lam0[n_occ - 1]))
        for run in runs:
            h = _history(run)
            ref = osp2.estimate_gap(h["sigma_c"], h["iderr"], h["layers"], e1, en, n, 1e-12)
            got = sp2.estimate_gap(dict(h, emin=e1, emax=en), n, "fp64")
            assert (ref is None) == (got is None), (ref, got)
            if ref is not None:
                compared += 1
                assert abs(got[0] - ref[0]) <= 1e-12 * max(1.0, abs(ref[0]))
                assert abs(got[1] - ref[1]) <= 1e-12 * max(1.0, abs(ref[1]))
    assert compared > 100


def test_estimate_argument_errors():
    L = sp2.lib()
    info = sp2.Info()
    ho, lu = ctypes.c_double(), ctypes.c_double()
    assert L.sp2_estimate_gap(None, 10, 0, ctypes.byref(ho), ctypes.byref(lu)) == sp2.SP2_EINVAL
    info.layers = 2
    info.emin, info.emax = -1.0, 1.0
    assert L.sp2_estimate_gap(ctypes.byref(info), 10, 0, ctypes.byref(ho), ctypes.byref(lu)) == sp2.SP2_EINVAL
    info.layers = 10                                   # no history values: no usable pair
    assert L.sp2_estimate_gap(ctypes.byref(info), 10, 0, ctypes.byref(ho), ctypes.byref(lu)) == sp2.SP2_EINVAL
    assert L.sp2_estimate_gap(ctypes.byref(info), 0, 0, ctypes.byref(ho), ctypes.byref(lu)) == sp2.SP2_EINVAL
    assert L.sp2_estimate_gap(ctypes.byref(info), 10, 7, ctypes.byref(ho), ctypes.byref(lu)) == sp2.SP2_EINVAL
