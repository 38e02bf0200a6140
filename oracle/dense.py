"""Dense brute-force references for tiny sizes.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

* `solve_dense`: explicit Kronecker-sum matrix + LU (N <= a few thousand).
* `solve_kron_eig`: full-tensor solve through per-mode eigendecompositions
  (N up to ~1e6), x = (x)_k V_k [ ((x)_k V_k^-1 b) / Lambda ].
* `sgmres_dense`: Alg. 1 (sGMRES) on explicit matrices, the reference for the
  reduction test "TT-sGMRES without truncation == sGMRES".

Pins: `solve_dense` is LAPACK; `solve_kron_eig` against `solve_dense`;
`sgmres_dense` with S = I and a full window against numpy's least squares on
the Krylov matrix (textbook GMRES) (tests/test_oracle_closed_form.py,
tests/test_oracle_solvers.py).
"""
from __future__ import annotations

from typing import List

import numpy as np

from .operators import dense_kron_sum


def solve_dense(terms: List[List[np.ndarray]], b_full: np.ndarray) -> np.ndarray:
    A = dense_kron_sum(terms)
    return np.linalg.solve(A, b_full.reshape(-1)).reshape(b_full.shape)


def solve_kron_eig(terms: List[List[np.ndarray]], b_full: np.ndarray) -> np.ndarray:
    d = b_full.ndim
    A = [sum(term[k] for term in terms) for k in range(d)]
    T = b_full
    lam = 0.0
    Vs = []
    for k, Ak in enumerate(A):
        w, V = np.linalg.eig(Ak)
        w, V = w.real, V.real
        Vs.append(V)
        T = np.moveaxis(np.tensordot(np.linalg.inv(V), T, axes=([1], [k])), 0, k)
        shape = [1] * d
        shape[k] = Ak.shape[0]
        lam = lam + w.reshape(shape)
    T = T / lam
    for k, V in enumerate(Vs):
        T = np.moveaxis(np.tensordot(V, T, axes=([1], [k])), 0, k)
    return T


def sgmres_dense(A: np.ndarray, b: np.ndarray, x0: np.ndarray, maxit: int, S: np.ndarray,
                 q: int, tol: float):
    """Alg. 1 (sGMRES): Arnoldi with orthogonalization against the last q vectors
    (modified Gram-Schmidt order), y = (S A V_k)^+ S r0, stop when
    ||W_k y - S r0|| <= ||S b|| tol.  Returns (x, info)."""
    r0 = b - A @ x0
    V = [r0 / np.linalg.norm(r0)]
    W = []
    Sr0 = S @ r0
    Sb = np.linalg.norm(S @ b)
    hist = []
    y = None
    for k in range(1, maxit + 1):
        vt = A @ V[k - 1]
        W.append(S @ vt)
        for i in range(max(1, k - q + 1), k + 1):
            h = vt @ V[i - 1]
            vt = vt - h * V[i - 1]
        hk = np.linalg.norm(vt)
        Wk = np.array(W).T
        y = np.linalg.lstsq(Wk, Sr0, rcond=None)[0]
        res = np.linalg.norm(Wk @ y - Sr0)
        hist.append(res / Sb)
        if res <= Sb * tol or hk == 0.0:
            break
        V.append(vt / hk)
    x = x0 + np.array(V[:len(y)]).T @ y
    return x, {"iterations": len(hist), "sketched_residuals": hist}
