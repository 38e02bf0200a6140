"""TT-matrix form of Kronecker-sum operators (Sec. 2.2 operator format; Sec. 4.1; Sec. 5.1).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

A Kronecker sum  sum_k I x .. x M_k x .. x I  acts on mode k with M_k.  A sum of
`m` such terms is written with m+1 "states" per bond: state 0 = no mode matrix
placed yet, state t+1 = the matrix of term t has been placed.  Core D_k
(shape (R, n, n, R)) has identity on (0,0) and (t+1,t+1) and the mode matrix of
term t on (0, t+1); the first core keeps only state 0 on its left, the last core
sums the states into one.  One term gives the rank-2 form of the Laplacian;
two terms give the rank-3 forms of the convection-diffusion and potential
operators.

Pins: `dense_kron_sum` is checked against explicit `np.kron` products and the
TT-matrix against `dense_kron_sum` entry by entry (tests/test_oracle_tt.py).
"""
from __future__ import annotations

from typing import List

import numpy as np


def tt_kron_sum(terms: List[List[np.ndarray]]) -> List[np.ndarray]:
    """TT-matrix cores of sum_t sum_k (I x .. x terms[t][k] x .. x I)."""
    m = len(terms)
    d = len(terms[0])
    R = m + 1
    cores = []
    for k in range(d):
        n = terms[0][k].shape[0]
        I = np.eye(n)
        if d == 1:
            D = np.zeros((1, n, n, 1))
            D[0, :, :, 0] = sum(terms[t][0] for t in range(m))
            cores.append(D)
            continue
        if k == 0:
            D = np.zeros((1, n, n, R))
            D[0, :, :, 0] = I
            for t in range(m):
                D[0, :, :, t + 1] = terms[t][k]
        elif k == d - 1:
            D = np.zeros((R, n, n, 1))
            D[0, :, :, 0] = sum(terms[t][k] for t in range(m))
            for t in range(m):
                D[t + 1, :, :, 0] = I
        else:
            D = np.zeros((R, n, n, R))
            D[0, :, :, 0] = I
            for t in range(m):
                D[0, :, :, t + 1] = terms[t][k]
                D[t + 1, :, :, t + 1] = I
        cores.append(D)
    return cores


def dense_kron_sum(terms: List[List[np.ndarray]]) -> np.ndarray:
    """Explicit N x N matrix (N = prod n_k) for tiny sizes; mode 0 is the slowest index."""
    d = len(terms[0])
    ns = [terms[0][k].shape[0] for k in range(d)]
    N = int(np.prod(ns))
    A = np.zeros((N, N))
    for term in terms:
        for k in range(d):
            M = np.ones((1, 1))
            for j in range(d):
                M = np.kron(M, term[k] if j == k else np.eye(ns[j]))
            A += M
    return A


def dense_from_tt_matrix(A: List[np.ndarray]) -> np.ndarray:
    """Dense matrix of a TT-matrix by contracting its cores (tiny sizes only)."""
    M = A[0][0]                                      # (m0, n0, R1)
    M = M.reshape(M.shape[0], M.shape[1], M.shape[2])
    rows, cols = M.shape[0], M.shape[1]
    for D in A[1:]:
        Rl, m, n, Rr = D.shape
        M = np.einsum('ijx,xaby->iajby', M, D).reshape(rows * m, cols * n, Rr)
        rows, cols = rows * m, cols * n
    return M[:, :, 0]


def tt_markov(Q: List[np.ndarray], J: np.ndarray, P: np.ndarray, rate: float) -> List[np.ndarray]:
    """TT-matrix of the synchronized Markov chain of Sec. 5.1.2:
        A = sum_k Q_k  +  rate sum_{k<d-1} (J_k x J_{k+1})  -  rate sum_{k<d-1} (P_k x P_{k+1})
    (each term acting on the named modes, identity elsewhere): the independent
    walks Q = (+)_k Q_k, the joint transitions W of neighbouring systems and the
    row-sum correction D = diag(W 1).  Four states per bond: 0 = nothing placed,
    1 = one term complete, 2 = a J of a pair placed, 3 = a P of a pair placed;
    a pair opened at mode k must close at mode k+1.  The bond rank is 4 for
    every d (the paper's remark that the rank grows with d describes a
    representation that adds the terms one by one)."""
    d = len(Q)
    n = Q[0].shape[0]
    I = np.eye(n)
    cores = []
    for k in range(d):
        D = np.zeros((4, n, n, 4))
        D[0, :, :, 0] = I
        D[1, :, :, 1] = I
        D[0, :, :, 1] = Q[k]
        D[0, :, :, 2] = rate * J
        D[0, :, :, 3] = -rate * P
        D[2, :, :, 1] = J
        D[3, :, :, 1] = P
        if k == 0:
            D = D[0:1]
        if k == d - 1:
            D = D[:, :, :, 1:2]
        cores.append(np.ascontiguousarray(D))
    return cores


def dense_markov(Q: List[np.ndarray], J: np.ndarray, P: np.ndarray, rate: float) -> np.ndarray:
    """Explicit matrix of tt_markov by Kronecker products (mode 0 slowest); tiny sizes."""
    d = len(Q)
    n = Q[0].shape[0]

    def place(mats):
        M = np.ones((1, 1))
        for k in range(d):
            M = np.kron(M, mats.get(k, np.eye(n)))
        return M
    A = sum(place({k: Q[k]}) for k in range(d))
    for k in range(d - 1):
        A = A + rate * place({k: J, k + 1: J}) - rate * place({k: P, k + 1: P})
    return A
