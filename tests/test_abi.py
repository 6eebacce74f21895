"""The C ABI library loads and exports every symbol that include/sp2.h declares, and its
host-only entry points (defaults, status strings, workspace sizing, argument checks
that return before any device work) behave as documented.  No GPU needed."""
import ctypes
import os
import re

import pytest

from paper_2101_06385_amd import sp2

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sp2.h")

pytestmark = pytest.mark.skipif(not os.path.exists(sp2.LIB_PATH), reason="libsp2.so not built")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sp2_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_entry_points():
    names = declared_functions()
    for want in ("sp2_density", "sp2_workspace_size", "sp2_default_options", "sp2_strerror", "sp2_query",
                 "sp2_square"):
        assert want in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(sp2.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_struct_layouts_match_the_c_compiler(tmp_path):
    """sizeof/offsetof of the ABI structs as the C compiler lays them out."""
    import shutil
    import subprocess

    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    src = tmp_path / "layout.c"
    src.write_text(
        '#include <stddef.h>\n#include <stdio.h>\n#include "sp2.h"\n'
        "int main(void){printf(\"%zu %zu %zu %zu %zu %zu %zu %zu %zu\\n\", sizeof(sp2_options), sizeof(sp2_info),"
        " offsetof(sp2_options, tile), offsetof(sp2_info, sigma), offsetof(sp2_info, iderr),"
        " offsetof(sp2_info, nx), offsetof(sp2_options, homo), offsetof(sp2_info, gap_violation),"
        " offsetof(sp2_info, sigma_c));return 0;}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    want = [ctypes.sizeof(sp2.Options), ctypes.sizeof(sp2.Info), sp2.Options.tile.offset,
            sp2.Info.sigma.offset, sp2.Info.iderr.offset, sp2.Info.nx.offset, sp2.Options.homo.offset,
            sp2.Info.gap_violation.offset, sp2.Info.sigma_c.offset]
    assert got == want


def test_defaults_and_strings():
    o = sp2.Options()
    sp2.lib().sp2_default_options(ctypes.byref(o))
    assert o.precision == sp2.FP16X2 and o.max_layers == 100 and o.refine == 1 and o.scale_log2 == -1
    assert o.eps == 0.0 and o.have_bounds == 0 and o.tile == 0
    assert o.accelerate == 0 and o.homo == 0.0 and o.lumo == 0.0
    for st in range(-6, 1):
        assert isinstance(sp2.strerror(st), str) and sp2.strerror(st)
    assert "gfx950" in sp2.version()


def test_split_workspaces_hold_padded_planes():
    # the half planes of an np x np matrix are stored with a row pitch of np + 64 halves
    L = sp2.lib()
    for n in (1000, 4096, 8192, 16384):
        np_ = L.sp2_square_padded(n, sp2.FP16X2, 0)
        assert np_ >= n
        assert L.sp2_square_workspace_size(n, sp2.FP16X2, 0, 0) >= 4 * np_ * (np_ + 64)
        full = sp2.workspace_size(n, sp2.options(precision="fp16x2"))
        assert full >= np_ * np_ * (2 * 4 + 2 * 8) + 4 * 2 * np_ * (np_ + 64)


def test_workspace_size_scales_with_n_and_precision():
    sizes = {}
    for p in ("fp64", "fp32", "fp16x2", "bf16x2"):
        o = sp2.options(precision=p)
        sizes[p] = [sp2.workspace_size(n, o) for n in (1, 100, 1000, 8192)]
        assert all(s > 0 for s in sizes[p])
        assert sizes[p] == sorted(sizes[p])
    np_ = 8192
    # split mode: two FP32 states + four half planes + FP64 refinement input and output
    assert sizes["fp16x2"][-1] >= np_ * np_ * (2 * 4 + 4 * 2 + 2 * 8)
    assert sp2.workspace_size(0, sp2.options()) == 0


def test_invalid_options_give_zero_workspace():
    assert sp2.workspace_size(100, sp2.options(max_layers=200)) == 0
    assert sp2.workspace_size(100, sp2.options(tile=96)) == 0
    assert sp2.workspace_size(100, sp2.options(precision="fp64", tile=256)) == 0
    assert sp2.workspace_size(100, sp2.options(bounds=(1.0, -1.0))) == 0
    assert sp2.workspace_size(100, sp2.options(precision="fp16x2", scale_log2=15)) == 0
    assert sp2.workspace_size(100, sp2.options(kernel=9)) == 0
    assert sp2.workspace_size(100, sp2.options(kernel=8)) > 0
    assert sp2.workspace_size(100, sp2.options(kernel=-1)) == 0
    assert sp2.workspace_size(100, sp2.options(kernel=7, tile=128)) > 0
    assert sp2.workspace_size(100, sp2.options(precision="fp64", kernel=6)) == 0
    assert sp2.workspace_size(100, sp2.options(precision="fp64", kernel=3)) > 0
    # accelerated layers need homo < lumo, both finite
    assert sp2.workspace_size(100, sp2.options(gap=(-1.0, 1.0))) > 0
    assert sp2.workspace_size(100, sp2.options(gap=(1.0, -1.0))) == 0
    assert sp2.workspace_size(100, sp2.options(gap=(0.5, 0.5))) == 0
    assert sp2.workspace_size(100, sp2.options(gap=(float("nan"), 1.0))) == 0


def test_argument_errors_return_before_device_work():
    L = sp2.lib()
    o = sp2.options()
    fake = ctypes.c_void_p(256)   # never dereferenced: every call below fails validation first
    cases = [
        dict(n=0, n_occ=0, ldh=1, ldd=1),
        dict(n=10, n_occ=-1, ldh=10, ldd=10),
        dict(n=10, n_occ=11, ldh=10, ldd=10),
        dict(n=10, n_occ=5, ldh=9, ldd=10),
        dict(n=10, n_occ=5, ldh=10, ldd=9),
    ]
    for c in cases:
        st = L.sp2_density(fake, c["ldh"], fake, c["ldd"], c["n"], c["n_occ"], 0.0, ctypes.byref(o), None,
                           fake, 1 << 40, None)
        assert st == sp2.SP2_EINVAL, c
    # null pointers
    assert L.sp2_density(None, 10, fake, 10, 10, 5, 0.0, ctypes.byref(o), None, fake, 1 << 40, None) == sp2.SP2_EINVAL
    # misaligned workspace
    assert L.sp2_density(fake, 10, fake, 10, 10, 5, 0.0, ctypes.byref(o), None, ctypes.c_void_p(260), 1 << 40,
                         None) == sp2.SP2_EINVAL
    # workspace too small
    assert L.sp2_density(fake, 10, fake, 10, 10, 5, 0.0, ctypes.byref(o), None, fake, 16, None) == sp2.SP2_ENOMEM
    # bad options
    bad = sp2.options(max_layers=500)
    assert L.sp2_density(fake, 10, fake, 10, 10, 5, 0.0, ctypes.byref(bad), None, fake, 1 << 40,
                         None) == sp2.SP2_EINVAL


def test_square_padding_helpers():
    L = sp2.lib()
    assert L.sp2_square_padded(300, sp2.FP16X2, 64) == 320
    assert L.sp2_square_padded(300, sp2.FP16X2, 256) == 512
    assert L.sp2_square_padded(8192, sp2.FP16X2, 0) == 8192
    assert L.sp2_square_workspace_size(300, sp2.FP16X2, 64, 0) > 4 * 320 * 320
    # stream-K buffers only where that schedule can run (split modes, tiles of 128 or 256)
    assert L.sp2_square_workspace_size(8192, sp2.FP16X2, 256, 2) > L.sp2_square_workspace_size(8192, sp2.FP16X2, 256, 1)
    assert L.sp2_square_workspace_size(8192, sp2.FP64, 128, 2) == L.sp2_square_workspace_size(8192, sp2.FP64, 128, 1)


def test_batched_workspace_and_argument_errors():
    L = sp2.lib()
    o = sp2.options()
    sizes = [64, 130, 700]
    total = sp2.batched_workspace_size(sizes, o)
    # per problem at least two FP32 state matrices, four half planes and two FP64 refinement buffers
    assert total >= sum(n * n * (2 * 4 + 4 * 2 + 2 * 8) for n in sizes)
    assert sp2.batched_workspace_size([], o) == 0
    assert sp2.batched_workspace_size([0, 10], o) == 0
    assert sp2.batched_workspace_size(sizes, sp2.options(precision="fp64")) == 0
    assert sp2.batched_workspace_size(sizes, sp2.options(bounds=(-1.0, 1.0))) == 0
    assert sp2.batched_workspace_size(sizes, sp2.options(gap=(-1.0, 1.0))) == 0
    fake = ctypes.c_void_p(256)
    P = ctypes.c_void_p * 1
    I = ctypes.c_int * 1
    ph, pd = P(256), P(256)

    def call(n, n_occ, ldh, ldd, work=1 << 40, ws=fake):
        return L.sp2_density_batched(1, ph, I(ldh), pd, I(ldd), I(n), I(n_occ), 0.0, ctypes.byref(o), None, 1,
                                     ws, work, None)

    assert call(10, 5, 9, 10) == sp2.SP2_EINVAL
    assert call(10, 5, 10, 9) == sp2.SP2_EINVAL
    assert call(10, 11, 10, 10) == sp2.SP2_EINVAL
    assert call(0, 0, 1, 1) == sp2.SP2_EINVAL
    assert call(10, 5, 10, 10, ws=ctypes.c_void_p(260)) == sp2.SP2_EINVAL
    assert call(10, 5, 10, 10, work=16) == sp2.SP2_ENOMEM
    assert L.sp2_density_batched(0, ph, I(10), pd, I(10), I(10), I(5), 0.0, ctypes.byref(o), None, 1, fake,
                                 1 << 40, None) == sp2.SP2_EINVAL
    D = ctypes.c_double * 1

    def call_gap(homo, lumo):
        return L.sp2_density_batched_gap(1, ph, I(10), pd, I(10), I(10), I(5), homo, lumo, 0.0, ctypes.byref(o), None,
                                         1, fake, 16, None)

    assert call_gap(D(1.0), D(-1.0)) == sp2.SP2_EINVAL          # homo >= lumo
    assert call_gap(D(float("nan")), D(1.0)) == sp2.SP2_EINVAL
    assert call_gap(None, D(1.0)) == sp2.SP2_EINVAL
    assert call_gap(D(-1.0), D(1.0)) == sp2.SP2_ENOMEM          # valid interval: reaches the size check


def test_autotune_sizes_and_argument_errors():
    L = sp2.lib()
    assert sp2.lib().sp2_autotune_workspace_size(0, sp2.FP16X2) == 0
    assert sp2.lib().sp2_autotune_workspace_size(1000, sp2.FP64) == 0
    w = sp2.lib().sp2_autotune_workspace_size(3000, sp2.FP16X2)
    assert w >= 2 * 4 * 3072 * 3072
    fake = ctypes.c_void_p(256)
    t, k, ms = ctypes.c_int(), ctypes.c_int(), ctypes.c_float()
    args = (ctypes.byref(t), ctypes.byref(k), ctypes.byref(ms))
    assert L.sp2_autotune(0, sp2.FP16X2, 3, *args, fake, 1 << 40, None) == sp2.SP2_EINVAL
    assert L.sp2_autotune(100, sp2.FP32, 3, *args, fake, 1 << 40, None) == sp2.SP2_EINVAL
    assert L.sp2_autotune(100, sp2.FP16X2, 0, *args, fake, 1 << 40, None) == sp2.SP2_EINVAL
    assert L.sp2_autotune(100, sp2.FP16X2, 3, *args, ctypes.c_void_p(260), 1 << 40, None) == sp2.SP2_EINVAL
    assert L.sp2_autotune(100, sp2.FP16X2, 3, *args, fake, 16, None) == sp2.SP2_ENOMEM
    sizes = (ctypes.c_int * 3)(256, 512, 640)
    o = sp2.options()
    bw = L.sp2_autotune_batched_workspace_size(3, sizes, ctypes.byref(o))
    o64 = sp2.options(tile=64)
    assert bw >= sp2.batched_workspace_size([256, 512, 640], o64)
    L.sp2_autotune_reset()


def test_static_entry_point_host_checks():
    """sp2_density_static rejects bad arguments (SP2_EINVAL) and problems whose workspace
    exceeds its scratch array (SP2_ENOMEM) before touching the device."""
    L = sp2.lib()
    o = sp2.options()
    fake = ctypes.c_void_p(256)   # never dereferenced
    limit = 40 << 20
    for prec in ("fp16x2", "bf16x2", "fp32", "fp64"):
        assert sp2.workspace_size(1024, sp2.options(prec)) <= limit, prec
    assert sp2.workspace_size(2048, o) > limit
    assert L.sp2_density_static(fake, 2048, fake, 2048, 2048, 100, 0.0, ctypes.byref(o), None, None) == sp2.SP2_ENOMEM
    assert L.sp2_density_static(fake, 10, fake, 10, 10, 11, 0.0, ctypes.byref(o), None, None) == sp2.SP2_EINVAL
    assert L.sp2_density_static(fake, 9, fake, 10, 10, 5, 0.0, ctypes.byref(o), None, None) == sp2.SP2_EINVAL
    assert L.sp2_density_static(None, 10, fake, 10, 10, 5, 0.0, ctypes.byref(o), None, None) == sp2.SP2_EINVAL
    bad = sp2.options(max_layers=500)
    assert L.sp2_density_static(fake, 10, fake, 10, 10, 5, 0.0, ctypes.byref(bad), None, None) == sp2.SP2_EINVAL


def test_net_checkpoint_default_keeps_every_layer_while_small():
    # ckpt_every = 0: every layer kept (K + 7 matrices) while that takes at most 8 GiB,
    # else checkpoints ceil(sqrt(K)) apart (ceil(K / c) + c + 6 matrices)
    f16 = sp2.FP16X2
    L = sp2.lib()
    for n, K in ((2048, 20), (200, 9)):
        assert L.sp2_net_workspace_size(n, K, f16, 0) == L.sp2_net_workspace_size(n, K, f16, 1)
        assert L.sp2_net_workspace_size(n, K, f16, 0) > L.sp2_net_workspace_size(n, K, f16, 5)
    m2 = 16384 * 16384 * 4
    assert (20 + 7) * m2 > 8 << 30
    assert L.sp2_net_workspace_size(16384, 20, f16, 0) == L.sp2_net_workspace_size(16384, 20, f16, 5)
    assert L.sp2_net_workspace_size(16384, 20, f16, 0) < 20 * m2
