"""Pins of oracle/gradient.py: dense LU loss and dense adjoint gradient on a tiny
parametric system; central finite differences of the closed-form loss; the
exponential sums for 1/z^p against the exact powers."""
import numpy as np
import pytest

import synthetic as syn
from oracle import gradient as og
from oracle import operators as oops
from oracle import tt as ott


def _dense_embed(M, k, ns):
    out = np.ones((1, 1))
    for j, n in enumerate(ns):
        out = np.kron(out, M if j == k else np.eye(n))
    return out


@pytest.mark.parametrize("p", [1, 2, 3])
def test_inverse_power_sums(p):
    zmin, zmax = 30.0, 2.0e5
    t, w = og.inv_power_nodes(zmin, zmax, p)
    z = np.geomspace(zmin, zmax, 2000)
    approx = (w[None, :] * np.exp(-np.outer(z, t))).sum(axis=1)
    assert np.max(np.abs(approx * z ** p - 1.0)) < 1e-11


def test_closed_form_against_dense_adjoint():
    d, n = 3, 5
    rng = np.random.default_rng(0)
    theta = rng.uniform(0.5, 2.0, size=d)
    L = syn.laplacian_1d(n)
    Ls = [th * L for th in theta]
    b = syn.gaussian_tt(rng, [n] * d, [1, 2, 2, 1])
    xt = syn.gaussian_tt(rng, [n] * d, [1, 2, 2, 1])
    A = oops.dense_kron_sum([Ls])
    bf, tf = ott.full(b).reshape(-1), ott.full(xt).reshape(-1)
    x = np.linalg.solve(A, bf)
    loss = np.sum((x - tf) ** 2)
    lam = np.linalg.solve(A.T, 2 * (x - tf))
    grad = np.array([-lam @ (_dense_embed(L, k, [n] * d) @ x) for k in range(d)])
    # the closed form takes the unscaled mode matrices and theta separately
    l_cf, g_cf = og.loss_and_grad(theta, [L] * d, b, xt)
    assert abs(l_cf - loss) <= 1e-10 * loss
    assert np.allclose(g_cf, grad, rtol=1e-9, atol=1e-14 * np.abs(grad).max())


def test_closed_form_against_finite_differences():
    d, n = 8, 64
    w = syn.config_c4(d, n)
    l, g = og.loss_and_grad(w["theta"], [w["L"]] * d, w["b"], w["x_target"])
    fd = og.fd_grad(w["theta"], [w["L"]] * d, w["b"], w["x_target"], 1e-4)
    assert np.allclose(g, fd, rtol=1e-6)
    assert l > 0
