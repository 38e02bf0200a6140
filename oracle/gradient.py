"""Closed-form loss and gradient for the parametric operator A(theta) = sum_k theta_k L_k.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

L_k acts on mode k only (I x .. x L_k x .. x I) and is symmetric with
eigendecomposition L_k = V_k diag(l_k) V_k^T.  In the eigenbasis (cores of b and
x_t multiplied by V_k^T in mode k: b^, xt^) the operator is diagonal with
Lambda_j = sum_k theta_k l_k(j_k), so x^ = b^ / Lambda and

  L(theta)       = ||x - x_t||^2 = sum_j b^_j^2 / Lambda_j^2 - 2 sum_j b^_j xt^_j / Lambda_j + ||x_t||^2
  dL/dtheta_k    = -2 [ sum_j b^_j^2 l_k(j_k) / Lambda_j^3  -  sum_j xt^_j b^_j l_k(j_k) / Lambda_j^2 ].

Each 1/Lambda^p is an exponential sum (1/z^p = (1/Gamma(p)) int t^(p-1) e^(-t z) dt,
t = e^u, trapezoid rule in u), so every sum above is a sum over quadrature nodes
of separable products, which factor core by core:
  sum_j A_j B_j prod_m g_m(j_m) = prod_m ( sum_i g_m(i) A_m[:, i, :] (x) B_m[:, i, :] ).

The same derivative is what an adjoint solve gives: with lambda = A^-T 2 (x - x_t),
dL/dtheta_k = -<lambda, L_k x>.

Pins (tests/test_oracle_gradient.py): dense LU loss and dense adjoint gradient on a
tiny system; central finite differences (step 1e-4) of the closed-form loss.
"""
from __future__ import annotations

import math
from typing import List

import numpy as np


def _eig(Ls):
    out = []
    for L in Ls:
        lam, V = np.linalg.eigh(L)
        out.append((lam, V))
    return out


def _hat(cores, eig):
    return [np.einsum('ij,aib->ajb', V, C) for C, (lam, V) in zip(cores, eig)]


def inv_power_nodes(zmin: float, zmax: float, p: int, h: float = 0.2, eps: float = 1e-17):
    """Nodes/weights with 1/z^p ~ sum_q w_q exp(-t_q z) on [zmin, zmax]."""
    u_lo = (math.log(eps) - math.log(zmax) * p) / p
    u_hi = math.log((40.0 + 12.0 * p) / zmin)
    u = np.arange(u_lo, u_hi + h, h)
    t = np.exp(u)
    w = h * t ** p / math.gamma(p)
    return t, w


def _chain(A, B, gs):
    """prod_m sum_i g_m(i) A_m[:, i, :] (x) B_m[:, i, :], contracted left to right."""
    v = np.ones((1, 1))
    for Am, Bm, g in zip(A, B, gs):
        M = np.einsum('i,aib,cie->acbe', g, Am, Bm)
        v = np.einsum('ac,acbe->be', v, M)
    return float(v[0, 0])


def loss_and_grad(theta, Ls: List[np.ndarray], b, xt):
    """Closed-form L(theta) and dL/dtheta (float64)."""
    theta = np.asarray(theta, dtype=np.float64)
    d = len(Ls)
    eig = _eig(Ls)
    bh = _hat(b, eig)
    th = _hat(xt, eig)
    zmin = sum(theta[k] * eig[k][0].min() for k in range(d))
    zmax = sum(theta[k] * eig[k][0].max() for k in range(d))
    t1, w1 = inv_power_nodes(zmin, zmax, 1)
    t2, w2 = inv_power_nodes(zmin, zmax, 2)
    t3, w3 = inv_power_nodes(zmin, zmax, 3)

    def expg(t, k_special=None):
        gs = []
        for m in range(d):
            lam = eig[m][0]
            g = np.exp(-t * theta[m] * lam)
            if m == k_special:
                g = g * lam
            gs.append(g)
        return gs

    bb2 = sum(w * _chain(bh, bh, expg(t)) for t, w in zip(t2, w2))
    bt1 = sum(w * _chain(bh, th, expg(t)) for t, w in zip(t1, w1))
    tt0 = _chain(th, th, [np.ones_like(e[0]) for e in eig])
    loss = bb2 - 2.0 * bt1 + tt0
    grad = np.zeros(d)
    for k in range(d):
        a3 = sum(w * _chain(bh, bh, expg(t, k)) for t, w in zip(t3, w3))
        a2 = sum(w * _chain(th, bh, expg(t, k)) for t, w in zip(t2, w2))
        grad[k] = -2.0 * (a3 - a2)
    return loss, grad


def loss_closed_form(theta, Ls, b, xt) -> float:
    return loss_and_grad(theta, Ls, b, xt)[0]


def fd_grad(theta, Ls, b, xt, step: float = 1e-4):
    """Central finite differences of the closed-form loss."""
    theta = np.asarray(theta, dtype=np.float64)
    g = np.zeros_like(theta)
    for k in range(len(theta)):
        tp = theta.copy()
        tm = theta.copy()
        tp[k] += step
        tm[k] -= step
        g[k] = (loss_closed_form(tp, Ls, b, xt) - loss_closed_form(tm, Ls, b, xt)) / (2 * step)
    return g
