"""Closed-form solutions of Kronecker-sum systems (independent of any Krylov iteration).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

* Pure Laplacian: the 1-D matrix (n+1)^2 tridiag(-1,2,-1) is diagonalized by the
  orthogonal, symmetric DST-I matrix V[i,j] = sqrt(2/(n+1)) sin(i j pi/(n+1)) with
  eigenvalues 4 (n+1)^2 sin^2(j pi / (2(n+1))), so A x = b is solved exactly in
  the full tensor by x = V^{(x)d} ((V^{(x)d} b) / Lambda), Lambda = sum of mode eigenvalues.
* General Kronecker sums A = sum_k A_k (diagonalizable A_k = V_k diag(l_k) V_k^-1):
  1/z is written as the integral of exp(-t z) over t > 0; with t = e^u and the
  trapezoid rule in u (step h), 1/z ~ sum_q w_q exp(-t_q z), which is the
  exponential-sum representation of Sec. 4.1.  Then
  x* ~ sum_q w_q (x)_k exp(-t_q A_k) b, a TT of rank (#terms) x rank(b).

Pins (tests/test_oracle_closed_form.py): DST eigenpairs against numpy.linalg.eigh;
full DST solve against a dense LU solve; max |z E(z) - 1| over the spectrum;
exponential-sum solution against the DST solution and against dense LU.
"""
from __future__ import annotations

from typing import List, Tuple

import numpy as np


def dst_matrix(n: int) -> np.ndarray:
    i = np.arange(1, n + 1)
    return np.sqrt(2.0 / (n + 1)) * np.sin(np.outer(i, i) * np.pi / (n + 1))


def laplace_eigs(n: int) -> np.ndarray:
    j = np.arange(1, n + 1)
    return 4.0 * (n + 1) ** 2 * np.sin(j * np.pi / (2.0 * (n + 1))) ** 2


def _mode_apply(T: np.ndarray, M: np.ndarray, k: int) -> np.ndarray:
    """Apply M to mode k of a dense tensor."""
    return np.moveaxis(np.tensordot(M, T, axes=([1], [k])), 0, k)


def laplace_solve_full(b: np.ndarray) -> np.ndarray:
    """Exact solution of (sum_k (n_k+1)^2 tridiag(-1,2,-1) acting on mode k) x = b, dense."""
    d = b.ndim
    T = b
    lam = 0.0
    for k in range(d):
        n = b.shape[k]
        T = _mode_apply(T, dst_matrix(n), k)
        shape = [1] * d
        shape[k] = n
        lam = lam + laplace_eigs(n).reshape(shape)
    T = T / lam
    for k in range(d):
        T = _mode_apply(T, dst_matrix(b.shape[k]), k)
    return T


def expsum_nodes(zmin: float, zmax: float, h: float = 0.3, eps: float = 1e-16) -> Tuple[np.ndarray, np.ndarray]:
    """Nodes t_q and weights w_q with 1/z ~ sum_q w_q exp(-t_q z) on [zmin, zmax].

    From 1/z = int_R e^u exp(-e^u z) du and the trapezoid rule with step h: the
    lower cut leaves an error ~ e^{u_lo} z_max, the upper one is double-
    exponentially small once e^{u_hi} z_min >= 40."""
    u_lo = np.log(eps / zmax)
    u_hi = np.log(40.0 / zmin)
    u = np.arange(u_lo, u_hi + h, h)
    t = np.exp(u)
    return t, h * t


def expsum_max_error(t: np.ndarray, w: np.ndarray, zmin: float, zmax: float, npts: int = 4000) -> float:
    z = np.geomspace(zmin, zmax, npts)
    E = (w[None, :] * np.exp(-np.outer(z, t))).sum(axis=1)
    return float(np.max(np.abs(z * E - 1.0)))


def mode_matrices(terms: List[List[np.ndarray]]) -> List[np.ndarray]:
    """A_k = sum over terms of the matrix acting on mode k."""
    d = len(terms[0])
    return [sum(term[k] for term in terms) for k in range(d)]


def kron_sum_solve_tt(terms: List[List[np.ndarray]], b: List[np.ndarray], h: float = 0.3):
    """Exponential-sum solution as a list of (weight, TT) pairs, x* ~ sum_q w_q x_q.

    x_q has cores exp(-t_q A_k) applied to mode k of the cores of b."""
    A = mode_matrices(terms)
    eig = []
    zmin, zmax = 0.0, 0.0
    for Ak in A:
        lam, V = np.linalg.eig(Ak)
        if np.max(np.abs(lam.imag)) > 1e-10 * np.max(np.abs(lam)):
            raise ValueError("complex spectrum: not covered by the real exponential sum")
        lam = lam.real
        V = V.real
        eig.append((lam, V, np.linalg.inv(V)))
        zmin += lam.min()
        zmax += lam.max()
    t, w = expsum_nodes(zmin, zmax, h)
    out = []
    for tq, wq in zip(t, w):
        cores = []
        for (lam, V, Vi), C in zip(eig, b):
            E = (V * np.exp(-tq * lam)) @ Vi
            cores.append(np.einsum('ij,ajb->aib', E, C))
        out.append((wq, cores))
    return out


def expsum_entry(sol, idx) -> float:
    total = 0.0
    for wq, cores in sol:
        v = np.ones((1, 1))
        for c, i in zip(cores, idx):
            v = v @ c[:, i, :]
        total += wq * v[0, 0]
    return total


def expsum_full(sol) -> np.ndarray:
    from .tt import full
    return sum(wq * full(c) for wq, c in sol)


def expsum_round(sol, tol: float = 1e-12, maxrank=None):
    """x* as one TT: the terms are summed in chunks with TT-SVD rounding in between."""
    from .tt import add, round_svd, scale
    acc = None
    for wq, cores in sol:
        term = scale(cores, wq)
        acc = term if acc is None else round_svd(add(acc, term), tol, maxrank)
    return acc
