"""Seeded synthetic Hamiltonians with the spectra of the benchmark workloads.

This module only draws inputs: eigenvalue spectra, Haar-distributed orthogonal
matrices and the symmetric matrices built from them.  It contains none of the
density-matrix arithmetic; both the CPU oracle and the GPU path receive the same
arrays from here.

Every Hamiltonian is H = Q diag(eps) Q^T with Q the orthogonal factor of the QR
decomposition of a seeded standard-normal matrix, sign-fixed by diag(R) so that
Q is Haar distributed.  The band edges next to the gap are pinned (the highest
occupied eigenvalue sits at the top of the occupied band, the lowest virtual one
at the bottom of the virtual band), so the stated gap is exact.  The paper uses
synthetic random Hamiltonians only (the 10x10 case of its convergence figure,
the 100x100 case of its acceleration figure); these generators stand in for the
unspecified matrices behind its throughput figure.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np


@dataclass
class Workload:
    """A synthetic problem: H (FP64, symmetric), its construction and occupation."""

    name: str
    n: int
    n_occ: int
    eps: np.ndarray            # eigenvalues, ascending, FP64
    q: Optional[np.ndarray]    # eigenvectors (columns), FP64, None if not built
    h: np.ndarray              # Hamiltonian, FP64, exactly symmetric
    homo: float = float("nan")
    lumo: float = float("nan")
    extra: dict = field(default_factory=dict)


def _band(rng, count, lo, hi, pin):
    """`count` values uniform in [lo, hi] with one of them pinned to `pin`."""
    if count <= 0:
        return np.zeros(0)
    vals = rng.uniform(lo, hi, size=count - 1)
    return np.concatenate([vals, [pin]])


def gapped_spectrum(rng, n, n_occ, occ_lo, homo, lumo, virt_hi):
    """Occupied band uniform in [occ_lo, homo], virtual band uniform in [lumo, virt_hi].

    The HOMO and LUMO values are pinned so the gap is exactly lumo - homo.
    Returned ascending.
    """
    occ = _band(rng, n_occ, occ_lo, homo, homo)
    virt = _band(rng, n - n_occ, lumo, virt_hi, lumo)
    return np.sort(np.concatenate([occ, virt]))


def haar_orthogonal(rng, n, device=None):
    """Haar-distributed orthogonal matrix: QR of a standard-normal matrix, sign-fixed.

    `device` is None for NumPy/LAPACK, or a torch device string to factorize there
    (the normal matrix is always drawn by the NumPy generator, so the draw is the same).
    """
    g = rng.standard_normal((n, n))
    if device is None:
        q, r = np.linalg.qr(g)
        return q * np.sign(np.diag(r))[None, :]
    import torch

    gt = torch.from_numpy(g).to(device)
    q, r = torch.linalg.qr(gt)
    q = q * torch.sign(torch.diagonal(r))[None, :]
    return q.cpu().numpy()


def symmetric_from_eigen(q, eps, device=None):
    """H = Q diag(eps) Q^T, then (H + H^T)/2 so that H is exactly symmetric."""
    if device is None:
        h = (q * eps[None, :]) @ q.T
        return 0.5 * (h + h.T)
    import torch

    qt = torch.from_numpy(q).to(device)
    et = torch.from_numpy(np.ascontiguousarray(eps)).to(device)
    h = (qt * et[None, :]) @ qt.T.contiguous()
    h = 0.5 * (h + h.T.contiguous())
    return h.cpu().numpy()


def _build(name, rng, eps, n_occ, homo, lumo, device=None, **extra):
    n = eps.shape[0]
    q = haar_orthogonal(rng, n, device)
    h = symmetric_from_eigen(q, eps, device)
    return Workload(name, n, n_occ, eps, q, h, homo, lumo, dict(extra))


def config1(seed=1000, n=256):
    """FP64 SP2 case: N=256, 128 occupied in [-20,-1] eV, 128 virtual in [1,20] eV (gap 2 eV)."""
    rng = np.random.default_rng(seed)
    n_occ = n // 2
    eps = gapped_spectrum(rng, n, n_occ, -20.0, -1.0, 1.0, 20.0)
    return _build("c1_fp64_n%d" % n, rng, eps, n_occ, -1.0, 1.0)


def config2(seed=2000, n=4096, device=None):
    """Mixed-precision case: N=4096, 1/4 occupied in [-30,-0.5], rest in [0.5,30] (gap 1 eV)."""
    rng = np.random.default_rng(seed)
    n_occ = n // 4
    eps = gapped_spectrum(rng, n, n_occ, -30.0, -0.5, 0.5, 30.0)
    return _build("c2_mixed_n%d" % n, rng, eps, n_occ, -0.5, 0.5, device)


def config3(seed=3000, n=8192, device=None):
    """Small-gap stress case: 25% occupation, uniform density on [-25,25] eV with a
    0.2 eV gap at the 25% quantile (HOMO -12.55, LUMO -12.35)."""
    rng = np.random.default_rng(seed + n)
    n_occ = n // 4
    eps = gapped_spectrum(rng, n, n_occ, -25.0, -12.55, -12.35, 25.0)
    return _build("c3_gap0.2_n%d" % n, rng, eps, n_occ, -12.55, -12.35, device)


def config4(seed=4000, count=64, n_min_blocks=4, n_max_blocks=48, device=None):
    """Batched case: `count` problems, N_i = 64*U{4..48}, occupation fraction U[0.2,0.5],
    gap U[0.5,3] eV centred at that quantile of [-25,25] eV."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = 64 * int(rng.integers(n_min_blocks, n_max_blocks + 1))
        f = float(rng.uniform(0.2, 0.5))
        gap = float(rng.uniform(0.5, 3.0))
        n_occ = int(round(f * n))
        centre = -25.0 + 50.0 * f
        homo, lumo = centre - 0.5 * gap, centre + 0.5 * gap
        eps = gapped_spectrum(rng, n, n_occ, -25.0, homo, lumo, 25.0)
        out.append(_build("c4_batch%d_n%d" % (i, n), rng, eps, n_occ, homo, lumo, device))
    return out


def config5(seed=5000, n=2048, device=None):
    """Finite-temperature network case: spectrum uniform in [-15,15] eV, mu=0, kT=0.2 eV."""
    rng = np.random.default_rng(seed)
    eps = np.sort(rng.uniform(-15.0, 15.0, size=n))
    w = _build("c5_net_n%d" % n, rng, eps, n // 2, float("nan"), float("nan"), device,
               mu=0.0, kT=0.2)
    return w


def small_random(seed=6000, n=10, n_occ=5):
    """Uniform random symmetric H with H_ij in [-1,1] (the paper's 10x10 convergence case)."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(-1.0, 1.0, size=(n, n))
    h = np.triu(a) + np.triu(a, 1).T
    return Workload("small_random_n%d" % n, n, n_occ, np.full(n, np.nan), None, h)


def gapped(seed, n, n_occ, occ_lo=-20.0, homo=-1.0, lumo=1.0, virt_hi=20.0, device=None):
    """Generic gapped Hamiltonian used by tests at arbitrary sizes."""
    rng = np.random.default_rng(seed)
    eps = gapped_spectrum(rng, n, n_occ, occ_lo, homo, lumo, virt_hi)
    return _build("gapped_n%d_occ%d" % (n, n_occ), rng, eps, n_occ, homo, lumo, device)
