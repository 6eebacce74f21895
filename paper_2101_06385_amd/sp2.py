"""ctypes binding of libsp2 (C ABI in include/sp2.h).

Argument marshalling only: every step of the density-matrix computation runs in the
HIP kernels of libsp2.  PyTorch supplies device memory and the current stream.  The
library is loaded on first use; if it has not been built this raises instead of
falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libsp2.so")

SP2_OK, SP2_EINVAL, SP2_ENONFINITE, SP2_ENOCONV, SP2_ENOTIDEMP, SP2_EDEVICE, SP2_ENOMEM = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ENONFINITE", -3: "ENOCONV", -4: "ENOTIDEMP", -5: "EDEVICE",
                -6: "ENOMEM"}
FP64, FP32, FP16X2, BF16X2 = 0, 1, 2, 3
PRECISIONS = {"fp64": FP64, "fp32": FP32, "fp16x2": FP16X2, "bf16x2": BF16X2}
MAX_LAYERS = 128


class Options(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int),
        ("max_layers", ctypes.c_int),
        ("eps", ctypes.c_double),
        ("have_bounds", ctypes.c_int),
        ("emin", ctypes.c_double),
        ("emax", ctypes.c_double),
        ("refine", ctypes.c_int),
        ("scale_log2", ctypes.c_int),
        ("want_energy", ctypes.c_int),
        ("tile", ctypes.c_int),
        ("kernel", ctypes.c_int),
        ("accelerate", ctypes.c_int),
        ("homo", ctypes.c_double),
        ("lumo", ctypes.c_double),
    ]


class Info(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int),
        ("layers", ctypes.c_int),
        ("converged", ctypes.c_int),
        ("first_sign", ctypes.c_int),
        ("n_padded", ctypes.c_int),
        ("tile", ctypes.c_int),
        ("kernel", ctypes.c_int),
        ("accelerated", ctypes.c_int),
        ("gap_violation", ctypes.c_int),
        ("reserved", ctypes.c_int),
        ("emin", ctypes.c_double),
        ("emax", ctypes.c_double),
        ("trace", ctypes.c_double),
        ("idem", ctypes.c_double),
        ("energy", ctypes.c_double),
        ("asym", ctypes.c_double),
        ("sigma", ctypes.c_byte * MAX_LAYERS),
        ("iderr", ctypes.c_double * MAX_LAYERS),
        ("ns", ctypes.c_double * MAX_LAYERS),
        ("nx", ctypes.c_double * MAX_LAYERS),
        ("sigma_c", ctypes.c_double * MAX_LAYERS),
    ]


class Timing(ctypes.Structure):
    _fields_ = [
        ("total_ms", ctypes.c_double),
        ("prep_ms", ctypes.c_double),
        ("loop_ms", ctypes.c_double),
        ("loop_active_ms", ctypes.c_double),
        ("refine_ms", ctypes.c_double),
        ("final_ms", ctypes.c_double),
        ("squarings", ctypes.c_int),
        ("pad", ctypes.c_int),
        ("square_ms", ctypes.c_float * MAX_LAYERS),
        ("refine_square_ms", ctypes.c_float * 2),
    ]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libsp2.so (after torch, so that the HIP runtime torch ships is the one bound)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libsp2.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
    import torch  # noqa: F401  (binds libamdhip64 first)

    L = ctypes.CDLL(LIB_PATH)
    c_int, c_double, c_size_t, c_void_p, c_float = (ctypes.c_int, ctypes.c_double, ctypes.c_size_t,
                                                     ctypes.c_void_p, ctypes.c_float)
    L.sp2_default_options.argtypes = [ctypes.POINTER(Options)]
    L.sp2_default_options.restype = None
    L.sp2_strerror.argtypes = [c_int]
    L.sp2_strerror.restype = ctypes.c_char_p
    L.sp2_version.argtypes = []
    L.sp2_version.restype = ctypes.c_char_p
    L.sp2_workspace_size.argtypes = [c_int, ctypes.POINTER(Options)]
    L.sp2_workspace_size.restype = c_size_t
    L.sp2_density.argtypes = [c_void_p, c_int, c_void_p, c_int, c_int, c_int, c_double, ctypes.POINTER(Options),
                              ctypes.POINTER(Info), c_void_p, c_size_t, c_void_p]
    L.sp2_density.restype = c_int
    L.sp2_density_static.argtypes = [c_void_p, c_int, c_void_p, c_int, c_int, c_int, c_double,
                                     ctypes.POINTER(Options), ctypes.POINTER(Info), c_void_p]
    L.sp2_density_static.restype = c_int
    L.sp2_density_timed.argtypes = L.sp2_density.argtypes + [ctypes.POINTER(Timing)]
    L.sp2_density_timed.restype = c_int
    L.sp2_query.argtypes = [c_void_p, c_int, ctypes.POINTER(Options), ctypes.POINTER(Info), c_void_p]
    L.sp2_query.restype = c_int
    L.sp2_square_padded.argtypes = [c_int, c_int, c_int]
    L.sp2_square_padded.restype = c_int
    L.sp2_square_workspace_size.argtypes = [c_int, c_int, c_int, c_int]
    L.sp2_square_workspace_size.restype = c_size_t
    L.sp2_square.argtypes = [c_void_p, c_void_p, c_int, c_int, c_int, c_int, c_int, c_float, c_float, c_float,
                             ctypes.POINTER(c_double), c_void_p, c_size_t, c_void_p]
    L.sp2_square.restype = c_int
    L.sp2_batched_workspace_size.argtypes = [c_int, ctypes.POINTER(c_int), ctypes.POINTER(Options)]
    L.sp2_batched_workspace_size.restype = c_size_t
    L.sp2_density_batched.argtypes = [c_int, ctypes.POINTER(c_void_p), ctypes.POINTER(c_int),
                                      ctypes.POINTER(c_void_p), ctypes.POINTER(c_int), ctypes.POINTER(c_int),
                                      ctypes.POINTER(c_int), c_double, ctypes.POINTER(Options),
                                      ctypes.POINTER(Info), c_int, c_void_p, c_size_t, c_void_p]
    L.sp2_density_batched.restype = c_int
    L.sp2_density_batched_gap.argtypes = [c_int, ctypes.POINTER(c_void_p), ctypes.POINTER(c_int),
                                          ctypes.POINTER(c_void_p), ctypes.POINTER(c_int), ctypes.POINTER(c_int),
                                          ctypes.POINTER(c_int), ctypes.POINTER(c_double), ctypes.POINTER(c_double),
                                          c_double, ctypes.POINTER(Options), ctypes.POINTER(Info), c_int, c_void_p,
                                          c_size_t, c_void_p]
    L.sp2_density_batched_gap.restype = c_int
    L.sp2_autotune_workspace_size.argtypes = [c_int, c_int]
    L.sp2_autotune_workspace_size.restype = c_size_t
    L.sp2_autotune.argtypes = [c_int, c_int, c_int, ctypes.POINTER(c_int), ctypes.POINTER(c_int),
                               ctypes.POINTER(c_float), c_void_p, c_size_t, c_void_p]
    L.sp2_autotune.restype = c_int
    L.sp2_autotune_batched_workspace_size.argtypes = [c_int, ctypes.POINTER(c_int), ctypes.POINTER(Options)]
    L.sp2_autotune_batched_workspace_size.restype = c_size_t
    L.sp2_autotune_batched.argtypes = [c_int, ctypes.POINTER(c_void_p), ctypes.POINTER(c_int),
                                       ctypes.POINTER(c_void_p), ctypes.POINTER(c_int), ctypes.POINTER(c_int),
                                       ctypes.POINTER(c_int), ctypes.POINTER(Options), ctypes.POINTER(c_int),
                                       ctypes.POINTER(c_float), c_void_p, c_size_t, c_void_p]
    L.sp2_autotune_batched.restype = c_int
    L.sp2_autotune_reset.argtypes = []
    L.sp2_autotune_reset.restype = None
    L.sp2_net_workspace_size.argtypes = [c_int, c_int, c_int, c_int]
    L.sp2_net_workspace_size.restype = c_size_t
    L.sp2_net_forward.argtypes = [c_void_p, c_int, c_int, c_int, c_void_p, c_void_p, c_void_p, c_int, c_int,
                                  c_void_p, c_int, c_void_p, c_size_t, c_void_p]
    L.sp2_net_forward.restype = c_int
    L.sp2_net_backward.argtypes = [c_void_p, c_int, c_int, c_int, c_void_p, c_void_p, c_void_p, c_int, c_int,
                                   c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]
    L.sp2_net_backward.restype = c_int
    pd = ctypes.POINTER(c_double)
    L.sp2_observable_workspace_size.argtypes = [c_int]
    L.sp2_observable_workspace_size.restype = c_size_t
    L.sp2_observable.argtypes = [c_void_p, c_int, c_void_p, c_int, c_int, pd, c_void_p, c_size_t, c_void_p]
    L.sp2_observable.restype = c_int
    L.sp2_estimate_gap.argtypes = [ctypes.POINTER(Info), c_int, c_int, pd, pd]
    L.sp2_estimate_gap.restype = c_int
    L.sp2_fermi_fit.argtypes = [c_int, c_double, c_double, c_double, c_double, c_int, c_int, pd, pd, pd]
    L.sp2_fermi_fit.restype = c_int
    L.sp2_fermi_workspace_size.argtypes = [c_int, ctypes.POINTER(Options)]
    L.sp2_fermi_workspace_size.restype = c_size_t
    L.sp2_fermi_apply.argtypes = [c_void_p, c_int, c_void_p, c_int, c_int, c_int, pd, pd, ctypes.POINTER(Options), pd,
                                  c_void_p, c_size_t, c_void_p]
    L.sp2_fermi_apply.restype = c_int
    L.sp2_spectral_bounds_workspace_size.argtypes = [c_int]
    L.sp2_spectral_bounds_workspace_size.restype = c_size_t
    L.sp2_spectral_bounds.argtypes = [c_void_p, c_int, c_int, pd, pd, c_void_p, c_size_t, c_void_p]
    L.sp2_spectral_bounds.restype = c_int
    _lib = L
    return L


def _prec(p) -> int:
    if isinstance(p, str):
        return PRECISIONS[p.lower()]
    return int(p)


def options(precision="fp16x2", max_layers=100, eps=0.0, bounds=None, refine=True, scale_log2=-1,
            want_energy=False, tile=0, kernel=0, gap=None) -> Options:
    """sp2_options; `gap` = (homo, lumo) selects accelerated layers (an interval inside the
    HOMO-LUMO gap of H)."""
    o = Options()
    lib().sp2_default_options(ctypes.byref(o))
    o.precision = _prec(precision)
    o.max_layers = int(max_layers)
    o.eps = float(eps)
    if bounds is not None:
        o.have_bounds = 1
        o.emin, o.emax = float(bounds[0]), float(bounds[1])
    o.refine = 1 if refine else 0
    o.scale_log2 = int(scale_log2)
    o.want_energy = 1 if want_energy else 0
    o.tile = int(tile)
    o.kernel = int(kernel)
    if gap is not None:
        o.accelerate = 1
        o.homo, o.lumo = float(gap[0]), float(gap[1])
    return o


def strerror(status: int) -> str:
    return lib().sp2_strerror(int(status)).decode()


def version() -> str:
    return lib().sp2_version().decode()


def workspace_size(n: int, opts: Optional[Options] = None) -> int:
    return int(lib().sp2_workspace_size(int(n), ctypes.byref(opts) if opts is not None else None))


def _stream_ptr(device, stream=None):
    import torch

    if stream is None:
        stream = torch.cuda.current_stream(device)
    return ctypes.c_void_p(stream.cuda_stream)


def alloc_workspace(nbytes: int, device):
    """Device bytes for the library (256-byte aligned view of a torch allocation)."""
    import torch

    buf = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % 256
    return buf[off:off + int(nbytes)]


def info_dict(info: Info) -> dict:
    m = max(0, min(int(info.layers) + 1, MAX_LAYERS))
    return {
        "status": int(info.status),
        "status_name": STATUS_NAMES.get(int(info.status), "?"),
        "layers": int(info.layers),
        "converged": bool(info.converged),
        "first_sign": int(info.first_sign),
        "n_padded": int(info.n_padded),
        "tile": int(info.tile),
        "kernel": int(info.kernel),
        "emin": float(info.emin),
        "emax": float(info.emax),
        "trace": float(info.trace),
        "idem": float(info.idem),
        "energy": float(info.energy),
        "asym": float(info.asym),
        "sigma": [int(info.sigma[i]) for i in range(m)],
        "iderr": [float(info.iderr[i]) for i in range(m)],
        "ns": [float(info.ns[i]) for i in range(m)],
        "nx": [float(info.nx[i]) for i in range(m)],
        "accelerated": int(info.accelerated),
        "gap_violation": int(info.gap_violation),
        "sigma_c": [float(info.sigma_c[i]) for i in range(m)],
    }


class SP2Error(RuntimeError):
    def __init__(self, status, where="sp2"):
        super().__init__("%s: %s (%d)" % (where, STATUS_NAMES.get(status, "?"), status))
        self.status = status


def timing_dict(t: Timing) -> dict:
    k = int(t.squarings)
    return {
        "total_ms": float(t.total_ms), "prep_ms": float(t.prep_ms), "loop_ms": float(t.loop_ms),
        "loop_active_ms": float(t.loop_active_ms), "refine_ms": float(t.refine_ms),
        "final_ms": float(t.final_ms), "squarings": k,
        "square_ms": [float(t.square_ms[i]) for i in range(MAX_LAYERS)],
        "refine_square_ms": [float(t.refine_square_ms[0]), float(t.refine_square_ms[1])],
    }


def density(h, n_occ: int, tol: float = 0.0, precision="fp16x2", max_layers=100, eps=0.0, bounds=None,
            refine=True, scale_log2=-1, want_energy=False, tile=0, kernel=0, out=None, workspace=None,
            sync=True, stream=None, timed=False, gap=None):
    """D = theta(mu I - H) with Tr D = n_occ (Alg. 1) for a symmetric FP64 CUDA tensor H.

    gap=(homo, lumo): accelerated layers (Sec. Accelerated Deep-NN SP2) from an interval
    that lies inside the HOMO-LUMO gap of H.

    Returns (D, info) with info a dict (sync=True) or None (sync=False, nothing is
    read back; use `query`).  Argument errors raise SP2Error; numerical outcomes are
    reported in info["status"].
    """
    import torch

    if not (isinstance(h, torch.Tensor) and h.is_cuda and h.dtype == torch.float64 and h.dim() == 2):
        raise TypeError("H must be a 2-D float64 CUDA tensor")
    n = h.shape[0]
    if h.shape[1] != n or h.stride(1) != 1:
        raise ValueError("H must be square with unit column stride")
    opts = options(precision, max_layers, eps, bounds, refine, scale_log2, want_energy, tile, kernel, gap)
    need = workspace_size(n, opts)
    if need == 0:
        raise SP2Error(SP2_EINVAL, "sp2_workspace_size")
    if workspace is None or workspace.numel() < need:
        workspace = alloc_workspace(need, h.device)
    if out is None:
        out = torch.empty((n, n), dtype=torch.float64, device=h.device)
    info = Info() if (sync or timed) else None
    args = (ctypes.c_void_p(h.data_ptr()), h.stride(0), ctypes.c_void_p(out.data_ptr()), out.stride(0), n,
            int(n_occ), float(tol), ctypes.byref(opts), ctypes.byref(info) if info is not None else None,
            ctypes.c_void_p(workspace.data_ptr()), workspace.numel(), _stream_ptr(h.device, stream))
    tm = Timing() if timed else None
    if timed:
        st = lib().sp2_density_timed(*args, ctypes.byref(tm))
    else:
        st = lib().sp2_density(*args)
    # host-side argument errors leave info untouched (n_padded == 0); the device-side
    # symmetry check also reports EINVAL but fills info and writes D
    if st in (SP2_EDEVICE, SP2_ENOMEM) or (st == SP2_EINVAL and (info is None or int(info.n_padded) == 0)):
        raise SP2Error(st, "sp2_density")
    if timed:
        return out, info_dict(info), timing_dict(tm)
    return out, (info_dict(info) if info is not None else None)


def density_static(h, n_occ: int, tol: float = 0.0, precision="fp16x2", max_layers=100, eps=0.0, bounds=None,
                   refine=True, scale_log2=-1, want_energy=False, tile=0, kernel=0, out=None, sync=True,
                   stream=None, gap=None):
    """sp2_density_static: the density() computation with the library's own per-device scratch
    memory instead of a workspace (for n up to the scratch size; calls on one device must
    not overlap).  Returns (D, info) like density()."""
    import torch

    if not (isinstance(h, torch.Tensor) and h.is_cuda and h.dtype == torch.float64 and h.dim() == 2):
        raise TypeError("H must be a 2-D float64 CUDA tensor")
    n = h.shape[0]
    if h.shape[1] != n or h.stride(1) != 1:
        raise ValueError("H must be square with unit column stride")
    opts = options(precision, max_layers, eps, bounds, refine, scale_log2, want_energy, tile, kernel, gap)
    if out is None:
        out = torch.empty((n, n), dtype=torch.float64, device=h.device)
    info = Info() if sync else None
    st = lib().sp2_density_static(ctypes.c_void_p(h.data_ptr()), h.stride(0), ctypes.c_void_p(out.data_ptr()),
                                  out.stride(0), n, int(n_occ), float(tol), ctypes.byref(opts),
                                  ctypes.byref(info) if info is not None else None, _stream_ptr(h.device, stream))
    if st in (SP2_EDEVICE, SP2_ENOMEM) or (st == SP2_EINVAL and (info is None or int(info.n_padded) == 0)):
        raise SP2Error(st, "sp2_density_static")
    return out, (info_dict(info) if info is not None else None)


def batched_workspace_size(sizes, opts: Optional[Options] = None) -> int:
    arr = (ctypes.c_int * len(sizes))(*[int(v) for v in sizes])
    return int(lib().sp2_batched_workspace_size(len(sizes), arr, ctypes.byref(opts) if opts is not None else None))


def density_batched(hs, n_occs, tol: float = 0.0, precision="fp16x2", max_layers=100, eps=0.0, scale_log2=-1,
                    want_energy=False, tile=0, use_graph=True, outs=None, workspace=None, stream=None, gaps=None):
    """D_i = theta(mu_i I - H_i) for a list of symmetric FP64 CUDA tensors of any sizes, all
    problems advanced together one layer per launch.  gaps: one (homo, lumo) per problem
    for accelerated layers (sp2_density_batched_gap).  Returns (list of D_i, list of info)."""
    import torch

    b = len(hs)
    if b == 0 or len(n_occs) != b:
        raise ValueError("need one n_occ per Hamiltonian")
    for h in hs:
        if not (isinstance(h, torch.Tensor) and h.is_cuda and h.dtype == torch.float64 and h.dim() == 2
                and h.shape[0] == h.shape[1] and h.stride(1) == 1):
            raise TypeError("every H must be a square 2-D float64 CUDA tensor with unit column stride")
    opts = options(precision, max_layers, eps, None, True, scale_log2, want_energy, tile, 0)
    sizes = [int(h.shape[0]) for h in hs]
    need = batched_workspace_size(sizes, opts)
    if need == 0:
        raise SP2Error(SP2_EINVAL, "sp2_batched_workspace_size")
    dev = hs[0].device
    if workspace is None or workspace.numel() < need:
        workspace = alloc_workspace(need, dev)
    if outs is None:
        outs = [torch.empty_like(h) for h in hs]
    infos = (Info * b)()
    ph = (ctypes.c_void_p * b)(*[h.data_ptr() for h in hs])
    pd = (ctypes.c_void_p * b)(*[d.data_ptr() for d in outs])
    lh = (ctypes.c_int * b)(*[h.stride(0) for h in hs])
    ld = (ctypes.c_int * b)(*[d.stride(0) for d in outs])
    nn = (ctypes.c_int * b)(*sizes)
    no = (ctypes.c_int * b)(*[int(v) for v in n_occs])
    if gaps is not None:
        if len(gaps) != b:
            raise ValueError("need one (homo, lumo) per Hamiltonian")
        ho = (ctypes.c_double * b)(*[float(g[0]) for g in gaps])
        lu = (ctypes.c_double * b)(*[float(g[1]) for g in gaps])
        st = lib().sp2_density_batched_gap(b, ph, lh, pd, ld, nn, no, ho, lu, float(tol), ctypes.byref(opts), infos,
                                           1 if use_graph else 0, ctypes.c_void_p(workspace.data_ptr()),
                                           workspace.numel(), _stream_ptr(dev, stream))
    else:
        st = lib().sp2_density_batched(b, ph, lh, pd, ld, nn, no, float(tol), ctypes.byref(opts), infos,
                                       1 if use_graph else 0, ctypes.c_void_p(workspace.data_ptr()),
                                       workspace.numel(), _stream_ptr(dev, stream))
    if st in (SP2_EDEVICE, SP2_ENOMEM) or (st == SP2_EINVAL and all(int(i.n_padded) == 0 for i in infos)):
        raise SP2Error(st, "sp2_density_batched")
    return outs, [info_dict(i) for i in infos]


def autotune(n: int, precision="fp16x2", reps: int = 3, device="cuda:0", stream=None) -> dict:
    """Measure every squaring schedule for an n x n problem on `device` and record the
    fastest for later automatic choices (see sp2_autotune)."""
    p = _prec(precision)
    need = int(lib().sp2_autotune_workspace_size(int(n), p))
    if need == 0:
        raise SP2Error(SP2_EINVAL, "sp2_autotune_workspace_size")
    ws = alloc_workspace(need, device)
    tile, kernel, ms = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_float(0.0)
    st = lib().sp2_autotune(int(n), p, int(reps), ctypes.byref(tile), ctypes.byref(kernel), ctypes.byref(ms),
                            ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(ws.device, stream))
    if st != SP2_OK:
        raise SP2Error(st, "sp2_autotune")
    return {"tile": tile.value, "kernel": kernel.value, "ms": ms.value}


def autotune_batched(hs, n_occs, precision="fp16x2", max_layers=100, stream=None) -> dict:
    """Time the batched solve of these problems with each grouped-kernel tile and record
    the faster one for this multiset of sizes (see sp2_autotune_batched)."""
    import torch

    b = len(hs)
    opts = options(precision, max_layers)
    sizes = (ctypes.c_int * b)(*[int(h.shape[0]) for h in hs])
    need = int(lib().sp2_autotune_batched_workspace_size(b, sizes, ctypes.byref(opts)))
    if need == 0:
        raise SP2Error(SP2_EINVAL, "sp2_autotune_batched_workspace_size")
    dev = hs[0].device
    ws = alloc_workspace(need, dev)
    outs = [torch.empty_like(h) for h in hs]
    ph = (ctypes.c_void_p * b)(*[h.data_ptr() for h in hs])
    pd = (ctypes.c_void_p * b)(*[d.data_ptr() for d in outs])
    lh = (ctypes.c_int * b)(*[h.stride(0) for h in hs])
    ld = (ctypes.c_int * b)(*[d.stride(0) for d in outs])
    no = (ctypes.c_int * b)(*[int(v) for v in n_occs])
    tile, ms = ctypes.c_int(0), ctypes.c_float(0.0)
    st = lib().sp2_autotune_batched(b, ph, lh, pd, ld, sizes, no, ctypes.byref(opts), ctypes.byref(tile),
                                    ctypes.byref(ms), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                    _stream_ptr(dev, stream))
    if st != SP2_OK:
        raise SP2Error(st, "sp2_autotune_batched")
    return {"tile": tile.value, "ms": ms.value}


def autotune_reset() -> None:
    lib().sp2_autotune_reset()


def query(workspace, n, precision="fp16x2", stream=None, device=None, **kw) -> dict:
    opts = options(precision, **kw)
    info = Info()
    lib().sp2_query(ctypes.c_void_p(workspace.data_ptr()), int(n), ctypes.byref(opts), ctypes.byref(info),
                    _stream_ptr(device or workspace.device, stream))
    return info_dict(info)


def square(x, alpha=1.0, beta=0.0, gamma=0.0, precision="fp16x2", tile=0, scale_log2=-1, workspace=None,
           want_sums=True, stream=None, kernel=0):
    """One layer Y = alpha X^2 + beta X + gamma I of a symmetric n x n CUDA tensor X (FP32 for
    the FP32/split modes, FP64 for FP64).  Returns (Y, (Tr Y, ||Y||_F^2) or None)."""
    import torch

    p = _prec(precision)
    n = x.shape[0]
    L = lib()
    np_ = L.sp2_square_padded(n, p, int(tile))
    dt = torch.float64 if p == FP64 else torch.float32
    if x.dtype != dt:
        raise TypeError("X must be %s for this precision" % dt)
    xp = torch.zeros((np_, np_), dtype=dt, device=x.device)
    xp[:n, :n] = x
    yp = torch.empty_like(xp)
    need = L.sp2_square_workspace_size(n, p, int(tile), int(kernel))
    if workspace is None or workspace.numel() < need:
        workspace = alloc_workspace(need, x.device)
    sums = (ctypes.c_double * 2)()
    st = L.sp2_square(ctypes.c_void_p(xp.data_ptr()), ctypes.c_void_p(yp.data_ptr()), n, p, int(tile),
                      int(kernel), int(scale_log2), float(alpha), float(beta), float(gamma), sums if want_sums else None,
                      ctypes.c_void_p(workspace.data_ptr()), workspace.numel(), _stream_ptr(x.device, stream))
    if st != SP2_OK:
        raise SP2Error(st, "sp2_square")
    return yp[:n, :n], ((sums[0], sums[1]) if want_sums else None)


# ------------------------------------------------------------------------------ network
def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def net_workspace_size(n, K, precision="fp16x2", ckpt_every=0) -> int:
    return int(lib().sp2_net_workspace_size(int(n), int(K), _prec(precision), int(ckpt_every)))


def net_forward(x0, w, b, c, precision="fp16x2", ckpt_every=0, workspace=None, stream=None):
    """X_K of the generalized-SP2 network for a symmetric FP32 CUDA tensor X_0 and FP32
    coefficient tensors (K,).  Returns (X_K, workspace); the workspace holds the checkpoints
    that net_backward needs."""
    import torch

    n, K = x0.shape[0], w.shape[0]
    for t in (x0, w, b, c):
        if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
            raise TypeError("network tensors must be contiguous float32 CUDA tensors")
    need = net_workspace_size(n, K, precision, ckpt_every)
    if need == 0:
        raise SP2Error(SP2_EINVAL, "sp2_net_workspace_size")
    if workspace is None or workspace.numel() < need:
        workspace = alloc_workspace(need, x0.device)
    xk = torch.empty_like(x0)
    st = lib().sp2_net_forward(_ptr(x0), x0.stride(0), n, K, _ptr(w), _ptr(b), _ptr(c), _prec(precision),
                               int(ckpt_every), _ptr(xk), xk.stride(0), _ptr(workspace), workspace.numel(),
                               _stream_ptr(x0.device, stream))
    if st != SP2_OK:
        raise SP2Error(st, "sp2_net_forward")
    return xk, workspace


def net_backward(gk, w, b, c, workspace, precision="fp16x2", ckpt_every=0, want_g0=True, stream=None):
    """Gradients (dW, dB, dc, G_0) for G_K = dL/dX_K, after net_forward with `workspace`."""
    import torch

    n, K = gk.shape[0], w.shape[0]
    gk = gk.contiguous()
    dw = torch.empty_like(w)
    db = torch.empty_like(b)
    dc = torch.empty_like(c)
    g0 = torch.empty_like(gk) if want_g0 else None
    st = lib().sp2_net_backward(_ptr(gk), gk.stride(0), n, K, _ptr(w), _ptr(b), _ptr(c), _prec(precision),
                                int(ckpt_every), _ptr(g0), gk.stride(0), _ptr(dw), _ptr(db), _ptr(dc),
                                _ptr(workspace), workspace.numel(), _stream_ptr(gk.device, stream))
    if st != SP2_OK:
        raise SP2Error(st, "sp2_net_backward")
    return dw, db, dc, g0


# ------------------------------------------------------------------ finite-temperature expansion
def fermi_fit(layers: int, mu: float, kT: float, bounds, grid: int = 1001, max_iter: int = 300):
    """Fit the L-layer expansion (Eq. general SP2 + read-out) to the Fermi function at (mu, kT)
    for spectral bounds `bounds` = (emin, emax) (see sp2_fermi_fit).  Returns (theta (L, 3),
    c (L + 1,), loss) as NumPy arrays / float."""
    import numpy as np

    theta = (ctypes.c_double * (3 * layers))()
    c = (ctypes.c_double * (layers + 1))()
    loss = ctypes.c_double()
    st = lib().sp2_fermi_fit(int(layers), float(mu), float(kT), float(bounds[0]), float(bounds[1]), int(grid),
                             int(max_iter), theta, c, ctypes.byref(loss))
    if st != SP2_OK:
        raise SP2Error(st, "sp2_fermi_fit")
    return np.array(theta[:]).reshape(layers, 3), np.array(c[:]), float(loss.value)


def spectral_bounds(h, stream=None):
    """FP64 Gershgorin bounds of a symmetric FP64 CUDA tensor, computed on the device."""
    n = h.shape[0]
    ws = alloc_workspace(lib().sp2_spectral_bounds_workspace_size(n), h.device)
    lo, hi = ctypes.c_double(), ctypes.c_double()
    st = lib().sp2_spectral_bounds(ctypes.c_void_p(h.data_ptr()), h.stride(0), n, ctypes.byref(lo), ctypes.byref(hi),
                                   ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(h.device, stream))
    if st != SP2_OK:
        raise SP2Error(st, "sp2_spectral_bounds")
    return float(lo.value), float(hi.value)


def fermi_workspace_size(n: int, bounds, precision="fp16x2", tile=0, kernel=0) -> int:
    o = options(precision, bounds=bounds, tile=tile, kernel=kernel)
    return int(lib().sp2_fermi_workspace_size(int(n), ctypes.byref(o)))


def fermi_apply(h, theta, c, bounds, precision="fp16x2", tile=0, kernel=0, out=None, workspace=None, stream=None,
                observables=True):
    """D = I - sum_i c_i X_i for the fitted network on the matrix H (see sp2_fermi_apply).
    Returns (D, (Tr D, ||D||_F^2, Tr[D H]) or None)."""
    import numpy as np
    import torch

    if not (isinstance(h, torch.Tensor) and h.is_cuda and h.dtype == torch.float64 and h.dim() == 2
            and h.shape[0] == h.shape[1] and h.stride(1) == 1):
        raise TypeError("H must be a square 2-D float64 CUDA tensor with unit column stride")
    theta = np.ascontiguousarray(np.asarray(theta, dtype=np.float64).ravel())
    c = np.ascontiguousarray(np.asarray(c, dtype=np.float64).ravel())
    layers = theta.size // 3
    if theta.size != 3 * layers or c.size != layers + 1:
        raise ValueError("theta must hold 3 L values and c L + 1")
    n = h.shape[0]
    o = options(precision, bounds=bounds, tile=tile, kernel=kernel)
    need = int(lib().sp2_fermi_workspace_size(n, ctypes.byref(o)))
    if need == 0:
        raise SP2Error(SP2_EINVAL, "sp2_fermi_workspace_size")
    if workspace is None or workspace.numel() < need:
        workspace = alloc_workspace(need, h.device)
    if out is None:
        out = torch.empty((n, n), dtype=torch.float64, device=h.device)
    pd = ctypes.POINTER(ctypes.c_double)
    obs = (ctypes.c_double * 3)() if observables else None
    st = lib().sp2_fermi_apply(ctypes.c_void_p(h.data_ptr()), h.stride(0), ctypes.c_void_p(out.data_ptr()),
                               out.stride(0), n, layers, theta.ctypes.data_as(pd), c.ctypes.data_as(pd),
                               ctypes.byref(o), obs, ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
                               _stream_ptr(h.device, stream))
    if st != SP2_OK:
        raise SP2Error(st, "sp2_fermi_apply")
    return out, (tuple(obs[:]) if obs is not None else None)


def estimate_gap(info: dict, n: int, precision="fp16x2"):
    """(homo, lumo) estimated from the history of a converged call (see sp2_estimate_gap), or
    None when the history holds no usable pair of layers."""
    raw = Info()
    raw.layers = int(info["layers"])
    raw.emin, raw.emax = float(info["emin"]), float(info["emax"])
    for i, v in enumerate(info["sigma_c"][:MAX_LAYERS]):
        raw.sigma_c[i] = float(v)
    for i, v in enumerate(info["iderr"][:MAX_LAYERS]):
        raw.iderr[i] = float(v)
    ho, lu = ctypes.c_double(), ctypes.c_double()
    st = lib().sp2_estimate_gap(ctypes.byref(raw), int(n), _prec(precision), ctypes.byref(ho), ctypes.byref(lu))
    if st != SP2_OK:
        return None
    return float(ho.value), float(lu.value)


def observable(d, a, stream=None):
    """(Tr D, ||D||_F^2, sum_ij D_ij A_ij) for FP64 CUDA tensors D and A (see sp2_observable)."""
    import torch

    n = d.shape[0]
    for t in (d, a):
        if not (t.is_cuda and t.dtype == torch.float64 and t.dim() == 2 and tuple(t.shape) == (n, n)
                and t.stride(1) == 1):
            raise TypeError("D and A must be square 2-D float64 CUDA tensors with unit column stride")
    ws = alloc_workspace(int(lib().sp2_observable_workspace_size(n)), d.device)
    out = (ctypes.c_double * 3)()
    st = lib().sp2_observable(ctypes.c_void_p(d.data_ptr()), d.stride(0), ctypes.c_void_p(a.data_ptr()), a.stride(0),
                              n, out, ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_ptr(d.device, stream))
    if st != SP2_OK:
        raise SP2Error(st, "sp2_observable")
    return tuple(out[:])
