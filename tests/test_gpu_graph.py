"""Repeated calls as in a molecular-dynamics loop: one asynchronous sp2_density call
captured in a HIP graph (through torch.cuda.graph on the library's stream) and replayed
for a sequence of Hamiltonians written into the same input buffer.  Every replay must
give the bit-identical D and the same per-call state as an eager call on that input;
eager work and synchronizations run between the replays."""
import time

import numpy as np
import pytest
import torch

from paper_2101_06385_amd import sp2, workloads as wl

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _hamiltonians(n, count, seed):
    return [wl.gapped(seed + i, n, n // 4, occ_lo=-20.0, homo=-0.5 - 0.1 * i, lumo=0.5, virt_hi=20.0)
            for i in range(count)]


@pytest.mark.parametrize("prec,n,accel", [("fp16x2", 1024, False), ("fp64", 600, False), ("fp16x2", 1024, True),
                                          ("bf16x2", 3000, False)])
def test_graph_replay_matches_eager_calls(prec, n, accel):
    ws_list = _hamiltonians(n, 3, 300 + n)
    gap = (-0.4, 0.5) if accel else None          # inside every case's gap [-0.5 - 0.1 i, 0.5]
    kw = dict(precision=prec, gap=gap)
    refs = []
    for w in ws_list:
        d, info = sp2.density(torch.from_numpy(w.h).to(DEV), w.n_occ, **kw)
        refs.append((d.cpu().numpy(), info))
        assert info["status"] == sp2.SP2_OK
        if accel:
            assert info["accelerated"] > 0
    static_h = torch.from_numpy(ws_list[0].h).to(DEV)
    static_d = torch.empty_like(static_h)
    opts = sp2.options(prec, gap=gap)
    ws = sp2.alloc_workspace(sp2.workspace_size(n, opts), static_h.device)
    n_occ = ws_list[0].n_occ
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        sp2.density(static_h, n_occ, out=static_d, workspace=ws, sync=False, **kw)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        sp2.density(static_h, n_occ, out=static_d, workspace=ws, sync=False, **kw)
    torch.cuda.synchronize()
    for rep in range(2):
        for w, (d_ref, i_ref) in zip(ws_list, refs):
            static_h.copy_(torch.from_numpy(w.h).to(DEV))
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert np.array_equal(static_d.cpu().numpy(), d_ref), (rep, w.name)
            q = sp2.query(ws, n, prec, gap=gap)
            assert q["status"] == i_ref["status"] and q["layers"] == i_ref["layers"]
            assert q["sigma"] == i_ref["sigma"] and q["trace"] == i_ref["trace"]
            # eager work of the program between replays
            x = torch.randn(256, 256, device=DEV)
            assert torch.isfinite(x @ x).all()
    # launch cost: eager asynchronous call vs replay of the captured one
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        sp2.density(static_h, n_occ, out=static_d, workspace=ws, sync=False, **kw)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(5):
        g.replay()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    print("%s n=%d: eager async call %.2f ms, graph replay %.2f ms" % (prec, n, (t1 - t0) / 5 * 1e3,
                                                                      (t2 - t1) / 5 * 1e3))
