"""Batched solve (many Hamiltonians of different sizes advanced together, one launch per
layer, optionally as one hipGraph): every problem must give exactly what the
single-problem path gives with the same tile and one-workgroup-per-tile schedule, and
the accuracy the oracle's eigendecomposition fixes (D = theta(mu I - H), Tr D = N_occ)."""
import numpy as np
import pytest
import torch

from oracle import dm
from paper_2101_06385_amd import sp2, workloads as wl

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _check_vs_oracle(w, d, info):
    ref = dm.dm_construct(w.q, w.eps, w.n_occ)
    got = d.cpu().numpy()
    fro = np.linalg.norm(got - ref)
    assert info["status"] == 0, info["status_name"]
    assert fro <= 1e-3 * np.sqrt(w.n), (w.name, fro)
    assert abs(np.trace(got) - w.n_occ) <= 1e-6, (w.name, np.trace(got) - w.n_occ)


@pytest.mark.parametrize("prec", ["fp16x2", "bf16x2", "fp32"])
def test_batched_matches_single_path_bitwise(prec):
    ws = [wl.gapped(40 + i, n, n // 3) for i, n in enumerate((64, 130, 200, 257, 384))]
    hs = [torch.from_numpy(w.h).to(DEV) for w in ws]
    outs, infos = sp2.density_batched(hs, [w.n_occ for w in ws], precision=prec, tile=64)
    for w, h, d, info in zip(ws, hs, outs, infos):
        d1, i1 = sp2.density(h, w.n_occ, precision=prec, tile=64, kernel=1)
        assert info["layers"] == i1["layers"] and info["sigma"] == i1["sigma"]
        assert torch.equal(d, d1), w.name
        if prec != "bf16x2":
            _check_vs_oracle(w, d, info)


@pytest.mark.parametrize("prec", ["fp16x2", "bf16x2"])
def test_batched_tile128_matches_single_path_bitwise(prec):
    """Grouped 128-tile launches (direct-to-LDS squaring, FP64 refinement kernel) against
    the single path with the same tile and one workgroup per tile."""
    ws = [wl.gapped(50 + i, n, n // 4) for i, n in enumerate((520, 700, 900))]
    hs = [torch.from_numpy(w.h).to(DEV) for w in ws]
    outs, infos = sp2.density_batched(hs, [w.n_occ for w in ws], precision=prec, tile=128)
    for w, h, d, info in zip(ws, hs, outs, infos):
        d1, i1 = sp2.density(h, w.n_occ, precision=prec, tile=128, kernel=1)
        assert info["layers"] == i1["layers"] and info["sigma"] == i1["sigma"]
        assert torch.equal(d, d1), w.name
        if prec == "fp16x2":
            _check_vs_oracle(w, d, info)


def test_batched_graph_and_stream_launch_agree():
    ws = [wl.gapped(60 + i, n, int(0.4 * n)) for i, n in enumerate((100, 300, 520))]
    hs = [torch.from_numpy(w.h).to(DEV) for w in ws]
    a, ia = sp2.density_batched(hs, [w.n_occ for w in ws], use_graph=True)
    b, ib = sp2.density_batched(hs, [w.n_occ for w in ws], use_graph=False)
    for x, y, p, q in zip(a, b, ia, ib):
        assert torch.equal(x, y) and p["layers"] == q["layers"]


def test_batched_config4_subset_vs_oracle():
    """The batched workload's generator (sizes 64*U{4..48}, mixed occupations and gaps):
    the first 12 problems, each checked against its eigendecomposition."""
    ws = wl.config4(count=12)
    hs = [torch.from_numpy(w.h).to(DEV) for w in ws]
    outs, infos = sp2.density_batched(hs, [w.n_occ for w in ws])
    for w, d, info in zip(ws, outs, infos):
        _check_vs_oracle(w, d, info)
        assert np.array_equal(d.cpu().numpy(), d.cpu().numpy().T)


def test_batched_with_trivial_and_single_problems():
    ws = [wl.gapped(70, 150, 50), wl.gapped(71, 90, 30)]
    hs = [torch.from_numpy(w.h).to(DEV) for w in ws]
    outs, infos = sp2.density_batched(hs + [hs[1]], [ws[0].n_occ, 0, 90])
    _check_vs_oracle(ws[0], outs[0], infos[0])
    assert torch.count_nonzero(outs[1]) == 0
    assert torch.equal(outs[2], torch.eye(90, dtype=torch.float64, device=DEV))
    one, io = sp2.density_batched(hs[:1], [ws[0].n_occ])
    assert torch.equal(one[0], outs[0])


def test_batched_strided_inputs_and_outputs():
    w = wl.gapped(80, 200, 70)
    big = torch.zeros((200, 256), dtype=torch.float64, device=DEV)
    big[:, :200] = torch.from_numpy(w.h)
    h = big[:, :200]
    dbig = torch.full((200, 240), 7.0, dtype=torch.float64, device=DEV)
    outs, infos = sp2.density_batched([h], [w.n_occ], outs=[dbig[:, :200]])
    _check_vs_oracle(w, outs[0], infos[0])
    assert torch.all(dbig[:, 200:] == 7.0)


def test_batched_rejects_fp64_and_bounds():
    h = torch.eye(64, dtype=torch.float64, device=DEV)
    with pytest.raises(sp2.SP2Error):
        sp2.density_batched([h], [10], precision="fp64")


@pytest.mark.parametrize("prec,tile,sizes", [("fp16x2", 64, (64, 130, 200, 257)), ("fp16x2", 128, (520, 700, 900)),
                                             ("bf16x2", 64, (90, 300))])
def test_batched_accelerated_matches_single_path_bitwise(prec, tile, sizes):
    """sp2_density_batched_gap: every problem's accelerated run (its own HOMO/LUMO interval)
    equals the single accelerated call with the same tile and schedule; a problem with an
    empty occupation rides along."""
    ws = [wl.gapped(70 + i, n, n // 3, occ_lo=-20.0, homo=-1.0 - 0.2 * i, lumo=1.0 + 0.1 * i, virt_hi=20.0)
          for i, n in enumerate(sizes)]
    hs = [torch.from_numpy(w.h).to(DEV) for w in ws]
    occ = [w.n_occ for w in ws]
    gaps = [(w.homo, w.lumo) for w in ws]
    extra = wl.gapped(79, 96, 30)
    hs.append(torch.from_numpy(extra.h).to(DEV))
    occ.append(0)
    gaps.append((-1.0, 1.0))
    outs, infos = sp2.density_batched(hs, occ, precision=prec, tile=tile, gaps=gaps)
    for w, h, d, info, g in zip(ws, hs, outs, infos, gaps):
        d1, i1 = sp2.density(h, w.n_occ, precision=prec, tile=tile, kernel=1, gap=g)
        assert info["accelerated"] == i1["accelerated"] > 0
        assert info["layers"] == i1["layers"] and info["sigma"] == i1["sigma"]
        assert info["sigma_c"] == i1["sigma_c"]
        assert torch.equal(d, d1), w.name
        if prec == "fp16x2":
            _check_vs_oracle(w, d, info)
    assert infos[-1]["status"] == 0 and torch.count_nonzero(outs[-1]).item() == 0


def test_batched_config4_full_vs_oracle():
    """All 64 problems of the batched workload (N_i = 64 U{4..48}), one call, each against its
    eigendecomposition."""
    ws = wl.config4(device=DEV)
    hs = [torch.from_numpy(w.h).to(DEV) for w in ws]
    outs, infos = sp2.density_batched(hs, [w.n_occ for w in ws])
    assert len(outs) == 64
    for w, d, info in zip(ws, outs, infos):
        _check_vs_oracle(w, d, info)


@pytest.mark.parametrize("max_layers", [30, 100])
def test_batched_layers_beyond_the_first_graph_part(max_layers):
    """The batched sequence runs layers 1..48 first and the rest only if a problem is still
    running: a problem with a 2e-4 eV gap needs more than 48 layers, the others stop
    earlier; with a cap of 30 the cap falls in the first part.  Each result must equal
    the single path's."""
    ws = [wl.gapped(70, 200, 90, homo=-1e-4, lumo=1e-4), wl.gapped(71, 130, 40), wl.gapped(72, 300, 150)]
    hs = [torch.from_numpy(w.h).to(DEV) for w in ws]
    for graph in (True, False):
        outs, infos = sp2.density_batched(hs, [w.n_occ for w in ws], tile=64, max_layers=max_layers,
                                          use_graph=graph)
        for w, h, d, info in zip(ws, hs, outs, infos):
            d1, i1 = sp2.density(h, w.n_occ, tile=64, kernel=1, max_layers=max_layers)
            assert info["layers"] == i1["layers"] and info["sigma"] == i1["sigma"], w.name
            assert info["status"] == i1["status"], w.name
            assert torch.equal(d, d1), w.name
        if max_layers == 100:
            assert infos[0]["layers"] > 48 and max(i["layers"] for i in infos[1:]) <= 48
        else:
            assert infos[0]["layers"] >= 29


def test_batched_cached_graphs_follow_the_layout():
    """Instantiated graphs are reused per (workspace, layout): alternating two batches of
    different sizes in one workspace, and then new matrices of the first batch's sizes,
    must give each call exactly what a fresh single call gives."""
    # sizes above 512, where the single path also refines on 128 tiles
    a = [wl.gapped(80 + i, n, n // 3) for i, n in enumerate((530, 600, 650))]
    b = [wl.gapped(90 + i, n, n // 2) for i, n in enumerate((520, 700))]
    c = [wl.gapped(95 + i, n, n // 4) for i, n in enumerate((530, 600, 650))]
    o = sp2.options("fp16x2", tile=128)
    ws = sp2.alloc_workspace(max(sp2.batched_workspace_size([w.n for w in s], o) for s in (a, b)), DEV)
    for batch in (a, b, a, c, b):
        hs = [torch.from_numpy(w.h).to(DEV) for w in batch]
        outs, infos = sp2.density_batched(hs, [w.n_occ for w in batch], tile=128, workspace=ws)
        for w, h, d, info in zip(batch, hs, outs, infos):
            d1, i1 = sp2.density(h, w.n_occ, tile=128, kernel=1)
            assert info["layers"] == i1["layers"], w.name
            assert torch.equal(d, d1), w.name
