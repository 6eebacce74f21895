"""The autotuner: its choice is a valid schedule, the automatic options then use it, the
results stay correct (vs the oracle's eigendecomposition), and a reset restores the
built-in rule."""
import numpy as np
import pytest
import torch

from oracle import dm
from paper_2101_06385_amd import sp2, workloads as wl

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def test_autotune_single_size_is_used_by_density():
    sp2.autotune_reset()
    w = wl.gapped(90, 3000, 1000)
    h = torch.from_numpy(w.h).to(DEV)
    _, before = sp2.density(h, w.n_occ)
    best = sp2.autotune(3000, "fp16x2", reps=2)
    assert best["tile"] in (64, 128, 256) and 1 <= best["kernel"] <= 7 and best["ms"] > 0
    d, info = sp2.density(h, w.n_occ)
    assert info["tile"] == best["tile"]
    assert info["kernel"] == best["kernel"] or best["kernel"] == 1
    ref = dm.dm_construct(w.q, w.eps, w.n_occ)
    assert info["status"] == 0
    assert np.linalg.norm(d.cpu().numpy() - ref) <= 1e-3 * np.sqrt(w.n)
    sp2.autotune_reset()
    _, after = sp2.density(h, w.n_occ)
    assert (after["tile"], after["kernel"]) == (before["tile"], before["kernel"])


def test_autotune_batched_tile_is_used():
    sp2.autotune_reset()
    ws = [wl.gapped(91 + i, n, n // 3) for i, n in enumerate((200, 450, 700))]
    hs = [torch.from_numpy(w.h).to(DEV) for w in ws]
    best = sp2.autotune_batched(hs, [w.n_occ for w in ws])
    assert best["tile"] in (64, 128)
    outs, infos = sp2.density_batched(hs, [w.n_occ for w in ws])
    for w, d, info in zip(ws, outs, infos):
        assert info["tile"] == best["tile"]
        ref = dm.dm_construct(w.q, w.eps, w.n_occ)
        assert np.linalg.norm(d.cpu().numpy() - ref) <= 1e-3 * np.sqrt(w.n)
    sp2.autotune_reset()
