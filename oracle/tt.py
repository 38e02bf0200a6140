"""TT format and TT arithmetic in plain float64 numpy (paper Sec. 2.2).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

A TT tensor is a list of d cores C_mu of shape (r_mu, n_mu, r_{mu+1}) with
r_0 = r_d = 1 (eq. tt-format; 0-based modes here).  A TT-matrix is a list of
cores D_mu of shape (R_mu, m_mu, n_mu, R_{mu+1}) (eq. operator tt-format).

Pins (tests/test_oracle_tt.py): `full`/`entry` against each other and against
hand-built rank-1 tensors; `matvec` against the dense Kronecker operator;
`dot`/`norm` against the full tensors; `round_svd` against exact recovery of a
minimal-rank TT at tol = 0, the error bound tol*||T|| and the SVD of the
unfoldings of a full tensor.
"""
from __future__ import annotations

from typing import List, Optional

import numpy as np

Cores = List[np.ndarray]


def ranks(x: Cores) -> List[int]:
    return [c.shape[0] for c in x] + [x[-1].shape[2]]


def sizes(x: Cores) -> List[int]:
    return [c.shape[1] for c in x]


def copy(x: Cores) -> Cores:
    return [np.array(c, dtype=np.float64, copy=True) for c in x]


def full(x: Cores) -> np.ndarray:
    """Dense tensor T[i_1..i_d] = C_1[1,i_1,:] C_2[:,i_2,:] ... C_d[:,i_d,1] (eq. tt-format)."""
    out = x[0][0]                                  # (n_1, r_1)
    for c in x[1:]:
        out = np.tensordot(out, c, axes=([out.ndim - 1], [0]))
    return out[..., 0]


def entry(x: Cores, idx) -> float:
    """One entry as the product of the matrices C_mu[:, i_mu, :]."""
    v = np.ones((1, 1))
    for c, i in zip(x, idx):
        v = v @ c[:, i, :]
    return float(v[0, 0])


def from_full(T: np.ndarray, tol: float = 0.0, maxrank: Optional[int] = None) -> Cores:
    """TT-SVD of a dense tensor (sequential truncated SVDs of the unfoldings)."""
    ns = T.shape
    d = len(ns)
    nrm = np.linalg.norm(T)
    delta = tol * nrm / np.sqrt(max(d - 1, 1))
    cores = []
    r = 1
    M = T.reshape(1, -1)
    for mu in range(d - 1):
        M = M.reshape(r * ns[mu], -1)
        U, s, Vt = np.linalg.svd(M, full_matrices=False)
        k = _trunc_rank(s, delta, maxrank)
        cores.append(U[:, :k].reshape(r, ns[mu], k))
        M = s[:k, None] * Vt[:k]
        r = k
    cores.append(M.reshape(r, ns[d - 1], 1))
    return cores


def matvec(A: Cores, x: Cores) -> Cores:
    """y = A x core by core:  G[(a,al), i, (b,be)] = sum_j D[al,i,j,be] C[a,j,b].

    The merged rank index has the vector rank outer and the operator rank inner,
    so the ranks of y are the products of the ranks of A and x (Sec. 2.2)."""
    out = []
    for D, C in zip(A, x):
        Rl, m, n, Rr = D.shape
        rl, n2, rr = C.shape
        assert n == n2
        G = np.einsum('xijy,ajb->axiby', D, C)
        out.append(G.reshape(rl * Rl, m, rr * Rr))
    return out


def transpose_op(A: Cores) -> Cores:
    """TT-matrix of the transposed operator: swap row and column mode indices."""
    return [np.ascontiguousarray(D.transpose(0, 2, 1, 3)) for D in A]


def dot(x: Cores, y: Cores) -> float:
    """<x, y> by a left-to-right sweep of environments E[a, p] (r_x x r_y)."""
    E = np.ones((1, 1))
    for X, Y in zip(x, y):
        E = np.einsum('ap,aib,pic->bc', E, X, Y, optimize=True)
    return float(E[0, 0])


def scale(x: Cores, a: float) -> Cores:
    out = copy(x)
    out[0] = out[0] * a
    return out


def add(x: Cores, y: Cores, a: float = 1.0, b: float = 1.0) -> Cores:
    """a x + b y with block cores; ranks add."""
    d = len(x)
    if d == 1:
        return [a * x[0] + b * y[0]]
    out = []
    for mu, (X, Y) in enumerate(zip(x, y)):
        rl1, n, rr1 = X.shape
        rl2, _, rr2 = Y.shape
        if mu == 0:
            C = np.concatenate([a * X, b * Y], axis=2)
        elif mu == d - 1:
            C = np.concatenate([X, Y], axis=0)
        else:
            C = np.zeros((rl1 + rl2, n, rr1 + rr2))
            C[:rl1, :, :rr1] = X
            C[rl1:, :, rr1:] = Y
        out.append(C)
    return out


def lin_comb(coeffs, vecs: List[Cores]) -> Cores:
    """sum_i coeffs[i] vecs[i] as one block TT (no rounding)."""
    acc = scale(vecs[0], coeffs[0])
    for c, v in zip(coeffs[1:], vecs[1:]):
        acc = add(acc, v, 1.0, c)
    return acc


def orthogonalize_left(x: Cores) -> Cores:
    """Left-orthogonal representation by Householder QR of each left unfolding."""
    out = copy(x)
    d = len(out)
    for mu in range(d - 1):
        rl, n, rr = out[mu].shape
        Q, R = np.linalg.qr(out[mu].reshape(rl * n, rr))
        k = Q.shape[1]
        out[mu] = Q.reshape(rl, n, k)
        out[mu + 1] = np.tensordot(R, out[mu + 1], axes=([1], [0]))
    return out


def orthogonalize_right(x: Cores) -> Cores:
    """Right-orthogonal representation: QR of the transposed right unfoldings."""
    out = copy(x)
    d = len(out)
    for mu in range(d - 1, 0, -1):
        rl, n, rr = out[mu].shape
        Q, R = np.linalg.qr(out[mu].reshape(rl, n * rr).T)
        k = Q.shape[1]
        out[mu] = Q.T.reshape(k, n, rr)
        out[mu - 1] = np.tensordot(out[mu - 1], R.T, axes=([2], [0]))
    return out


def norm(x: Cores) -> float:
    """Frobenius norm through orthogonalization (no Gram-matrix cancellation)."""
    y = orthogonalize_left(x)
    return float(np.linalg.norm(y[-1]))


def _trunc_rank(s: np.ndarray, delta: float, maxrank: Optional[int]) -> int:
    """Smallest k with sqrt(sum_{i>=k} s_i^2) <= delta, at least 1, then capped."""
    tail = np.sqrt(np.cumsum((s ** 2)[::-1]))[::-1]    # tail[k] = ||s[k:]||
    k = len(s)
    for j in range(len(s)):
        if tail[j] <= delta:
            k = j
            break
    k = max(k, 1)
    if maxrank is not None and maxrank > 0:
        k = min(k, maxrank)
    return k


def round_svd(x: Cores, tol: float, maxrank: Optional[int] = None) -> Cores:
    """Round(T, tol): TT-SVD rounding (Sec. 2.2; Alg. 2).

    Right-to-left QR orthogonalization, then a left-to-right sweep of truncated
    SVDs of the left unfoldings with the per-bond threshold
    delta = tol * ||T||_F / sqrt(d-1); the kept rank at each bond is the smallest
    one whose discarded tail is <= delta, capped at maxrank (maxrank overrides tol).
    The result satisfies ||T - Round(T)|| <= tol ||T|| when no cap is active."""
    d = len(x)
    y = orthogonalize_right(x)
    if d == 1:
        return y
    nrm = float(np.linalg.norm(y[0]))
    if nrm == 0.0:
        return [np.zeros((1, c.shape[1], 1)) for c in y]
    delta = tol * nrm / np.sqrt(d - 1)
    for mu in range(d - 1):
        rl, n, rr = y[mu].shape
        U, s, Vt = np.linalg.svd(y[mu].reshape(rl * n, rr), full_matrices=False)
        k = _trunc_rank(s, delta, maxrank)
        y[mu] = U[:, :k].reshape(rl, n, k)
        y[mu + 1] = np.tensordot(s[:k, None] * Vt[:k], y[mu + 1], axes=([1], [0]))
    return y
