"""Pins of oracle/solvers.py: reductions to dense sGMRES / textbook GMRES on tiny
systems, closed-form solutions, lucky breakdown, monotone sketched residual."""
import numpy as np
import pytest

import synthetic as syn
from oracle import closed_form as cf
from oracle import dense
from oracle import operators as ops
from oracle import sketch as sk
from oracle import solvers
from oracle import tt


def _tiny_system(seed=0, n=5, d=3):
    terms = [[syn.laplacian_1d(n)] * d, [syn.upwind_1d(n, 0.1)] + [np.zeros((n, n))] * (d - 1)]
    rng = np.random.default_rng(seed)
    b = syn.gaussian_tt(rng, [n] * d, [1, 2, 2, 1])
    return terms, b, rng


def test_dense_sgmres_with_identity_sketch_is_gmres():
    terms, b, rng = _tiny_system()
    A = ops.dense_kron_sum(terms)
    bf = tt.full(b).reshape(-1)
    N = len(bf)
    k = 7
    x, info = dense.sgmres_dense(A, bf, np.zeros(N), k, np.eye(N), k, 0.0)
    # textbook GMRES: minimize ||b - A x|| over the Krylov space K_k(A, b)
    K = np.array([np.linalg.matrix_power(A, j) @ bf for j in range(k)]).T
    Q, _ = np.linalg.qr(K)
    c = np.linalg.lstsq(A @ Q, bf, rcond=None)[0]
    res_gmres = np.linalg.norm(bf - A @ Q @ c) / np.linalg.norm(bf)
    assert abs(info["sketched_residuals"][-1] - res_gmres) <= 1e-8 * res_gmres + 1e-15
    assert np.allclose(x, Q @ c, rtol=1e-8, atol=1e-12 * np.abs(x).max())


@pytest.mark.parametrize("rounding", ["svd", "stta"])
def test_tt_sgmres_without_truncation_equals_dense_sgmres(rounding):
    n, d = 5, 3
    terms, b, rng = _tiny_system(1, n, d)
    A = ops.tt_kron_sum(terms)
    S = syn.kr_factors(rng, 24, [n] * d)
    rx, rho = syn.stta_ranks([n] * d, 25, 5)          # full target ranks: STTA is exact
    X = syn.tt_drm(rng, [n] * d, rx, 1, d)
    Y = syn.tt_drm(rng, [n] * d, rho, 0, d - 1)
    k = 8
    x, info = solvers.tt_sgmres(A, b, S, X, Y, maxit=k, tol=1e-30, q=k, round_tol=1e-14,
                                rounding=rounding, fixed_iterations=k, final_tol=1e-14)
    Ad = ops.dense_kron_sum(terms)
    bf = tt.full(b).reshape(-1)
    xd, infod = dense.sgmres_dense(Ad, bf, np.zeros_like(bf), k, sk.kr_dense(S), k, 0.0)
    assert np.allclose(info["sketched_residuals"], infod["sketched_residuals"], rtol=1e-6)
    assert np.linalg.norm(tt.full(x).reshape(-1) - xd) <= 1e-7 * np.linalg.norm(xd)


def test_tt_gmres_without_truncation_equals_dense_gmres():
    terms, b, rng = _tiny_system(2)
    A = ops.tt_kron_sum(terms)
    x, info = solvers.tt_gmres(A, b, 6, 1e-30, max_round=1e-14, final_tol=1e-14)
    Ad = ops.dense_kron_sum(terms)
    bf = tt.full(b).reshape(-1)
    N = len(bf)
    xd, infod = dense.sgmres_dense(Ad, bf, np.zeros(N), 6, np.eye(N), 6, 0.0)
    assert np.allclose(info["residuals"], infod["sketched_residuals"], rtol=1e-7)
    assert np.linalg.norm(tt.full(x).reshape(-1) - xd) <= 1e-8 * np.linalg.norm(xd)


def test_lucky_breakdown_on_eigenvector_rhs():
    n, d = 8, 4
    V = cf.dst_matrix(n)
    b = [V[:, 1].reshape(1, n, 1).copy() for _ in range(d)]
    terms = [[syn.laplacian_1d(n)] * d]
    A = ops.tt_kron_sum(terms)
    rng = np.random.default_rng(3)
    S = syn.kr_factors(rng, 20, [n] * d)
    rx, rho = syn.stta_ranks([n] * d, 8, 4)
    X = syn.tt_drm(rng, [n] * d, rx, 1, d)
    Y = syn.tt_drm(rng, [n] * d, rho, 0, d - 1)
    x, info = solvers.tt_sgmres(A, b, S, X, Y, maxit=10, tol=1e-6, q=1, round_tol=1e-8)
    assert info["iterations"] == 1
    lam = d * cf.laplace_eigs(n)[1]
    assert np.allclose(tt.full(x), tt.full(b) / lam, rtol=1e-9, atol=1e-14)


@pytest.mark.slow
def test_c1_converges_to_closed_form():
    w = syn.config_c1()
    A = ops.tt_kron_sum(w.terms)
    x, info = solvers.tt_sgmres(A, w.b, w.S, w.X, w.Y, maxit=w.maxit, tol=w.tol, q=w.q,
                                round_tol=w.round_tol, maxrank=None, stop_safety=w.stop_safety,
                                restart=w.restart)
    assert info["true_residual"] <= w.tol
    xe = cf.laplace_solve_full(tt.full(w.b))
    assert np.linalg.norm(tt.full(x) - xe) <= 1e-5 * np.linalg.norm(xe)
    # sketched residual is non-increasing inside each restart cycle (W only gains columns)
    sr = info["sketched_residuals"]
    for c in range(info["cycles"]):
        seg = sr[c * w.restart:(c + 1) * w.restart]
        assert all(b <= a * (1 + 1e-10) for a, b in zip(seg, seg[1:]))
    # the exact solution is invariant under i_k -> n-1-i_k (b and A are); x is within tolerance
    F = tt.full(x)
    assert np.linalg.norm(F - F[::-1, ::-1, ::-1, ::-1, ::-1]) <= 1e-5 * np.linalg.norm(F)
