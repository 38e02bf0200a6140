"""Exponential-sum right preconditioning (Sec. 4.1) in plain float64 numpy.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The dominant part of the operator is a Kronecker sum  M = sum_k (I x .. x M_k x .. x I)
and the preconditioner is the exponential-sum approximation of its inverse,
  P^{-1} = E(M) = sum_j alpha_j (x)_k exp(-beta_j M_k),   1/z ~ E(z) = sum_j alpha_j exp(-beta_j z),
so applying it to a TT sums zeta mode-multiplied copies of the tensor (ranks grow
by at most zeta; Sec. 4.1).

Coefficients (the paper takes them from an integral representation of 1/z):
  1/z = int_R exp(u - e^u z) du  (substitute t = e^u in 1/z = int_0^inf e^{-t z} dt),
discretized by the trapezoid rule with step h on [u_lo, u_hi]:
  beta_j = exp(u_j), alpha_j = h exp(u_j),  u_j = u_lo + j h.
For a relative accuracy `tol` of z E(z) on [zmin, zmax]:
  * lower cut: the dropped mass gives a relative error 1 - exp(-e^{u_lo} z) <= e^{u_lo} zmax,
    so u_lo = log(tol / (4 zmax));
  * upper cut: it gives exp(-e^{u_hi} z) <= exp(-e^{u_hi} zmin), so
    u_hi = log(log(4 / tol) / zmin);
  * step: the trapezoid error of this integrand decays like exp(-c / h) with c
    about 7 (measured over spectra of condition 1e2..1e5), so h = 6.5 / log(2 / tol).
The number of terms is zeta = ceil((u_hi - u_lo) / h) + 1, growing like
log(zmax / zmin) log(1 / tol).

Pins (tests/test_oracle_precond.py): max |z E(z) - 1| <= tol on a dense grid of
[zmin, zmax] for several intervals and tolerances; the TT application against the
dense operator sum_j alpha_j kron_k expm(-beta_j M_k); E(M) against the dense
inverse of the Kronecker sum on a tiny grid.
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

import numpy as np
import scipy.linalg

from . import tt as ttm

Cores = List[np.ndarray]


def expsum_coefficients(zmin: float, zmax: float, tol: float) -> Tuple[np.ndarray, np.ndarray]:
    """(alpha, beta) with |z E(z) - 1| <= tol for z in [zmin, zmax], 0 < zmin <= zmax."""
    if not (0.0 < zmin <= zmax) or not (0.0 < tol < 1.0):
        raise ValueError("need 0 < zmin <= zmax and 0 < tol < 1")
    u_lo = np.log(tol / (4.0 * zmax))
    u_hi = np.log(np.log(4.0 / tol) / zmin)
    h = 6.5 / np.log(2.0 / tol)
    zeta = int(np.ceil((u_hi - u_lo) / h)) + 1
    u = u_lo + h * np.arange(zeta)
    return h * np.exp(u), np.exp(u)


def expsum_eval(alpha: np.ndarray, beta: np.ndarray, z: np.ndarray) -> np.ndarray:
    """E(z) = sum_j alpha_j exp(-beta_j z)."""
    z = np.asarray(z, dtype=np.float64)
    return (alpha[None, :] * np.exp(-np.outer(z.reshape(-1), beta))).sum(axis=1).reshape(z.shape)


def mode_exponentials(beta: Sequence[float], mats: Sequence[np.ndarray]) -> List[List[np.ndarray]]:
    """E[j][k] = expm(-beta_j M_k) (scaling-and-squaring Pade of scipy)."""
    return [[scipy.linalg.expm(-bj * M) for M in mats] for bj in beta]


def precond_terms(alpha, E, x: Cores) -> List[Cores]:
    """The zeta TTs alpha_j (x)_k E[j][k] x whose sum is P^{-1} x (mode products
    keep the ranks of x; alpha_j is folded into the first core)."""
    out = []
    for aj, Ej in zip(alpha, E):
        cores = [np.einsum('ij,ajb->aib', Ek, C) for Ek, C in zip(Ej, x)]
        cores[0] = aj * cores[0]
        out.append(cores)
    return out


def apply_precond(alpha, E, x: Cores, tol: float, maxrank=None) -> Cores:
    """P^{-1} x as one TT: the zeta terms summed as a block TT, then TT-SVD
    rounding at relative tolerance tol (optionally capped)."""
    terms = precond_terms(alpha, E, x)
    return ttm.round_svd(ttm.lin_comb([1.0] * len(terms), terms), tol, maxrank)


def dense_precond(alpha, E) -> np.ndarray:
    """Explicit sum_j alpha_j kron_k E[j][k] (mode 0 slowest), tiny sizes only."""
    P = None
    for aj, Ej in zip(alpha, E):
        K = np.ones((1, 1))
        for Ek in Ej:
            K = np.kron(K, Ek)
        P = aj * K if P is None else P + aj * K
    return P
