"""Structured sketches: Khatri-Rao OSE (Sec. 3.1) and STTA (Sec. 3.3).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Khatri-Rao sketch: row j of S is the Kronecker product of the j-th rows of the
factors S_k, so (S x)_j = prod_mu ( sum_i S_mu[j,i] C_mu[:, i, :] ), a product
of r x r matrices evaluated left to right.

STTA (streaming TT approximation, the two-sided randomized rounding of Sec. 3.3):
with Gaussian TT-DRMs Y (left, ranks rho) and X (right, ranks r_X),
  left partial  L_b = Y_{<=b}^T C_{<=b}      (rho_b x t_b),   L_0 = 1
  right partial R_b = C_{>b}^T  X_{>b}       (t_b x rX_b),    R_d = 1
  Psi_mu[p, i, q] = sum_{a,c} L_mu[p, a] C_mu[a, i, c] R_{mu+1}[c, q]
                  = ((Y_{<=mu-1}^T x I) T_{<=mu} X_{>mu}) reshaped
  Omega_b = L_b R_b = Y_{<=b}^T T_{<=b} X_{>b}
and the recovered cores are  C^_0 = Psi_0,  C^_mu = Omega_mu^+ Psi_mu (right
unfolding).  The sketches are linear in the tensor, so the sketch of a linear
combination is the same combination of sketches (streaming sums).

Pins (tests/test_oracle_sketch.py): the KR sketch against the explicit s x N
matrix; E||Sx||^2 = ||x||^2 over many draws; STTA exact recovery when the
target ranks are at least the TT ranks; linearity of the sketches; invariance
of the recovered tensor to rescaling X and Y; Psi/Omega against the explicit
interface matrices of the DRMs on a tiny tensor.
"""
from __future__ import annotations

from typing import List, Optional, Tuple

import numpy as np

from . import tt as ttm

Cores = List[np.ndarray]


def kr_sketch(S: List[np.ndarray], x: Cores) -> np.ndarray:
    """(S x)_j for every sketch row j, as a left-to-right chain of row vectors P[j, :]."""
    s = S[0].shape[0]
    P = np.ones((s, 1))
    for Smu, C in zip(S, x):
        P = np.einsum('ja,ji,aib->jb', P, Smu, C, optimize=True)
    return P[:, 0]


def kr_dense(S: List[np.ndarray]) -> np.ndarray:
    """Explicit s x N Khatri-Rao matrix (row j = kron of the j-th factor rows); tiny sizes."""
    s = S[0].shape[0]
    rows = []
    for j in range(s):
        r = np.ones(1)
        for Smu in S:
            r = np.kron(r, Smu[j])
        rows.append(r)
    return np.array(rows)


def left_partials(x: Cores, Y: Cores) -> List[np.ndarray]:
    """L_b for b = 0..d-1 (L_0 = 1), L_{mu+1}[p, c] = sum Y_mu[p', i, p] L_mu[p', a] C_mu[a, i, c]."""
    d = len(x)
    L = [np.ones((1, 1))]
    for mu in range(d - 1):
        L.append(np.einsum('xip,xa,aic->pc', Y[mu], L[mu], x[mu], optimize=True))
    return L


def right_partials(x: Cores, X: Cores) -> List[np.ndarray]:
    """R_b for b = 1..d (R_d = 1), R_mu[a, q'] = sum C_mu[a, i, c] R_{mu+1}[c, q] X_mu[q', i, q].

    X holds the DRM cores of modes 1..d-1, so the core of mode mu is X[mu-1].
    Returned as a list indexed by bond with R[0] = None."""
    d = len(x)
    R = [None] * (d + 1)
    R[d] = np.ones((1, 1))
    for mu in range(d - 1, 0, -1):
        R[mu] = np.einsum('aic,cq,yiq->ay', x[mu], R[mu + 1], X[mu - 1], optimize=True)
    return R


def stta_sketch(x: Cores, X: Cores, Y: Cores) -> Tuple[List[np.ndarray], List[np.ndarray]]:
    """STTA_sketch: the core sketches Psi_mu (mu = 0..d-1) and the bond sketches
    Omega_b (b = 1..d-1, returned as a list of length d-1)."""
    d = len(x)
    L = left_partials(x, Y)
    R = right_partials(x, X)
    Psi = [np.einsum('pa,aic,cq->piq', L[mu], x[mu], R[mu + 1], optimize=True) for mu in range(d)]
    Omega = [L[b] @ R[b] for b in range(1, d)]
    return Psi, Omega


def pinv(M: np.ndarray, rcond: float) -> np.ndarray:
    """Moore-Penrose pseudo-inverse by SVD, dropping singular values below rcond * s_max."""
    U, s, Vt = np.linalg.svd(M, full_matrices=False)
    if s.size == 0 or s[0] == 0.0:
        return np.zeros((M.shape[1], M.shape[0]))
    keep = s > rcond * s[0]
    return (Vt[keep].T / s[keep]) @ U[:, keep].T


def stta_recover(Psi: List[np.ndarray], Omega: List[np.ndarray], rcond: float = 1e-12) -> Cores:
    """STTA_recover: C^_0 = Psi_0, C^_mu = Omega_mu^+ Psi_mu (right unfolding)."""
    d = len(Psi)
    cores = [np.array(Psi[0], copy=True)]
    for mu in range(1, d):
        rho, n, q = Psi[mu].shape
        Om = Omega[mu - 1]
        C = pinv(Om, rcond) @ Psi[mu].reshape(rho, n * q)
        cores.append(C.reshape(Om.shape[1], n, q))
    return cores


def lin_comb_sketches(coeffs, sketches) -> Tuple[List[np.ndarray], List[np.ndarray]]:
    """sum_i coeffs[i] * (Psi^(i), Omega^(i)) bond by bond (streaming sum)."""
    Psi = [coeffs[0] * p for p in sketches[0][0]]
    Omega = [coeffs[0] * o for o in sketches[0][1]]
    for c, (P, O) in zip(coeffs[1:], sketches[1:]):
        Psi = [a + c * p for a, p in zip(Psi, P)]
        Omega = [a + c * o for a, o in zip(Omega, O)]
    return Psi, Omega


def round_rand(x: Cores, X: Cores, Y: Cores, tol: float, maxrank: Optional[int] = None,
               rcond: float = 1e-12) -> Cores:
    """Randomized rounding: STTA sketch + recover at the sketch ranks, then TT-SVD
    of the small recovered tensor at `tol` (relative) with rank cap `maxrank`."""
    Psi, Omega = stta_sketch(x, X, Y)
    return ttm.round_svd(stta_recover(Psi, Omega, rcond), tol, maxrank)
