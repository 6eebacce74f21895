"""Exact density matrices by diagonalization (test infrastructure, CPU FP64).

Eq. 1 defines the finite-temperature density matrix D = (exp(beta(H - mu I)) + I)^-1,
Eq. 3 its zero-temperature limit theta(mu I - H), and Eqs. 4-6 evaluate either one
in the eigenbasis of H: D = Q f(E) Q^T with mu chosen so that Tr D = N_occ.
"""
from __future__ import annotations

import numpy as np
from scipy.special import expit


def dm_eigh(h: np.ndarray, n_occ: int) -> np.ndarray:
    """Zero-temperature D = Q theta(mu - E) Q^T (Eqs. 4, 6) with mu in the gap above
    the n_occ-th lowest eigenvalue: the projector on the n_occ lowest eigenvectors.

    Unique only when eigenvalue n_occ is strictly below eigenvalue n_occ+1.
    """
    h = np.asarray(h, dtype=np.float64)
    _, v = np.linalg.eigh(h)
    vo = v[:, :n_occ]
    return vo @ vo.T


def dm_construct(q: np.ndarray, eps: np.ndarray, n_occ: int) -> np.ndarray:
    """Same projector, for a Hamiltonian built as Q diag(eps) Q^T: no eigensolver needed.

    The occupied columns are those of the n_occ lowest values of eps.
    """
    order = np.argsort(eps, kind="stable")
    qo = np.asarray(q, dtype=np.float64)[:, order[:n_occ]]
    return qo @ qo.T


def dm_rows(q: np.ndarray, eps: np.ndarray, n_occ: int, rows) -> np.ndarray:
    """Selected rows of dm_construct, computed one by one (for sampled checks at large N)."""
    order = np.argsort(eps, kind="stable")
    qo = np.asarray(q, dtype=np.float64)[:, order[:n_occ]]
    return qo[np.asarray(rows)] @ qo.T


def fermi_dirac(eps: np.ndarray, mu: float, kT: float) -> np.ndarray:
    """Occupation f(e) = 1/(1 + exp((e - mu)/kT)) of Eq. 1 on the eigenvalues."""
    return expit(-(np.asarray(eps, dtype=np.float64) - mu) / kT)


def dm_fermi(q: np.ndarray, eps: np.ndarray, mu: float, kT: float) -> np.ndarray:
    """Finite-temperature D = Q f(E) Q^T (Eq. 5) for H = Q diag(eps) Q^T."""
    q = np.asarray(q, dtype=np.float64)
    return (q * fermi_dirac(eps, mu, kT)[None, :]) @ q.T


def fermi_rescaled(x: np.ndarray, beta: float = 40.0) -> np.ndarray:
    """The rescaled Fermi function F(x) = 1/(exp(beta(x - 1/2)) + 1) of Eq. fermi."""
    return expit(-beta * (np.asarray(x, dtype=np.float64) - 0.5))
