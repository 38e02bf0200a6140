"""Pins of oracle/precond.py (exponential-sum preconditioner, Sec. 4.1), of the
preconditioned (Alg. 5) and whitened (Sec. 3.4) forms of oracle/solvers.py, and
of the Markov-chain operator of Sec. 5.1.2 (oracle/operators.py)."""
import numpy as np
import pytest
import scipy.linalg

import synthetic as syn
from oracle import closed_form as cf
from oracle import dense
from oracle import operators as ops
from oracle import precond as pc
from oracle import sketch as sk
from oracle import solvers
from oracle import tt


@pytest.mark.parametrize("zmin,zmax", [(1.0, 100.0), (9.87, 6.6e4), (2.0e2, 1.33e6), (0.5, 3.0e5)])
@pytest.mark.parametrize("tol", [1e-1, 1e-2, 1e-4, 1e-8])
def test_expsum_accuracy_on_interval(zmin, zmax, tol):
    a, b = pc.expsum_coefficients(zmin, zmax, tol)
    z = np.geomspace(zmin, zmax, 20001)
    err = np.max(np.abs(z * pc.expsum_eval(a, b, z) - 1.0))
    assert err <= tol, err
    # terms grow like log(zmax/zmin) log(1/tol): a handful at tol 0.1, ~100 at 1e-8
    assert len(a) <= 4 + 0.25 * np.log(4 * zmax / (tol * zmin)) * np.log(2 / tol), len(a)


def test_expsum_inverse_of_kron_sum_dense():
    # E(M) ~ M^{-1} for a Kronecker sum: eigenvalues z E(z) within tol of 1
    n, d, tol = 5, 3, 1e-3
    L = syn.laplacian_1d(n)
    lam = cf.laplace_eigs(n)
    a, b = pc.expsum_coefficients(d * lam.min(), d * lam.max(), tol)
    E = pc.mode_exponentials(b, [L] * d)
    Pinv = pc.dense_precond(a, E)
    M = ops.dense_kron_sum([[L] * d])
    ev = np.linalg.eigvals(M @ Pinv)
    assert np.max(np.abs(ev - 1.0)) <= tol
    # each mode factor is the matrix exponential (against the eigendecomposition)
    w, V = np.linalg.eigh(L)
    assert np.allclose(E[2][1], (V * np.exp(-b[2] * w)) @ V.T, rtol=1e-10, atol=1e-14)


def test_precond_application_on_tt_matches_dense():
    n, d = 4, 3
    rng = np.random.default_rng(21)
    mats = [syn.convdiff_1d(n, K=1.0, w=2.0) + 0.5 * np.eye(n) for _ in range(d)]
    a, b = pc.expsum_coefficients(1.0, 200.0, 1e-2)
    E = pc.mode_exponentials(b, mats)
    x = syn.gaussian_tt(rng, [n] * d, [1, 3, 2, 1])
    y = pc.apply_precond(a, E, x, 1e-14)
    yd = pc.dense_precond(a, E) @ tt.full(x).reshape(-1)
    assert np.allclose(tt.full(y).reshape(-1), yd, rtol=1e-11, atol=1e-13 * np.abs(yd).max())
    # ranks grow by at most zeta
    assert max(tt.ranks(y)) <= len(a) * 3


def _sketch_set(rng, ns, s, cap, over=20):
    d = len(ns)
    S = syn.kr_factors(rng, s, ns)
    rx, rho = syn.stta_ranks(ns, cap, over)
    return S, syn.tt_drm(rng, ns, rx, 1, d), syn.tt_drm(rng, ns, rho, 0, d - 1)


def test_identity_preconditioner_reduces_to_alg4():
    # zeta = 1, alpha = 1, beta = 0: P^{-1} = I, Alg. 5 is Alg. 4 step for step
    n, d = 6, 3
    rng = np.random.default_rng(22)
    terms = [[syn.laplacian_1d(n)] * d, [syn.upwind_1d(n, 0.1)] + [np.zeros((n, n))] * (d - 1)]
    A = ops.tt_kron_sum(terms)
    b = syn.gaussian_tt(rng, [n] * d, [1, 2, 2, 1])
    S, X, Y = _sketch_set(rng, [n] * d, 40, 36)
    kw = dict(maxit=12, tol=1e-8, q=1, round_tol=1e-10)
    x1, i1 = solvers.tt_sgmres(A, b, S, X, Y, **kw)
    E = pc.mode_exponentials([0.0], [np.zeros((n, n))] * d)
    x2, i2 = solvers.tt_sgmres(A, b, S, X, Y, precond=(np.array([1.0]), E), **kw)
    assert np.allclose(i1["sketched_residuals"], i2["sketched_residuals"], rtol=1e-9)
    assert np.linalg.norm(tt.full(x1) - tt.full(x2)) <= 1e-9 * np.linalg.norm(tt.full(x1))


def test_preconditioned_laplacian_converges_fast_to_dst():
    n, d, tol = 16, 4, 1e-6
    rng = np.random.default_rng(23)
    L = syn.laplacian_1d(n)
    A = ops.tt_kron_sum([[L] * d])
    b = syn.gaussian_tt(rng, [n] * d, [1, 2, 2, 2, 1])
    S, X, Y = _sketch_set(rng, [n] * d, 40, 64)
    lam = cf.laplace_eigs(n)
    a, be = pc.expsum_coefficients(d * lam.min(), d * lam.max(), 1e-2)
    E = pc.mode_exponentials(be, [L] * d)
    x, info = solvers.tt_sgmres(A, b, S, X, Y, maxit=20, tol=tol, q=1, round_tol=1e-9, final_tol=1e-9,
                                precond=(a, E))
    assert info["true_residual"] <= tol
    assert info["iterations"] <= 6, info["iterations"]     # unpreconditioned: ~40
    xe = cf.laplace_solve_full(tt.full(b))
    assert np.linalg.norm(tt.full(x) - xe) <= 1e-6 * np.linalg.norm(xe)


@pytest.mark.slow
def test_preconditioned_convdiff_d5_n128_four_iterations():
    """Sec. 5.3.1: on the convection-diffusion problem with d = 5 the preconditioned
    iteration converges in 4 steps (zeta = 17, tol 1e-8 with the sketched
    residual held to 0.1 tol).  Here n = 128 and maxrank 30, the paper's cap."""
    n, d, tol = 128, 5, 1e-8
    A1 = syn.convdiff_1d(n)
    f = syn.gauss_source_1d(n)
    b = [f.reshape(1, n, 1).copy() for _ in range(d)]
    A = ops.tt_kron_sum([[A1] * d])
    rng = np.random.default_rng(24)
    S, X, Y = _sketch_set(rng, [n] * d, 40, 40)
    ev = np.linalg.eigvals(A1).real
    a, be = pc.expsum_coefficients(d * ev.min(), d * ev.max(), 1e-3)
    E = pc.mode_exponentials(be, [A1] * d)
    x, info = solvers.tt_sgmres(A, b, S, X, Y, maxit=20, tol=tol, q=1, round_tol=1e-9, final_tol=1e-10,
                                maxrank=30, stop_safety=0.1, precond=(a, E))
    assert info["true_residual"] <= tol, info["true_residual"]
    assert info["iterations"] <= 6, info["iterations"]


def test_whitening_without_truncation_equals_pseudo_inverse():
    # exact STTA (full target ranks), no rounding and a full window: the
    # sketched Arnoldi relation is exact and both least-squares forms minimize
    # the same ||S A V_k y - S r0||
    n, d = 5, 3
    rng = np.random.default_rng(25)
    terms = [[syn.laplacian_1d(n)] * d, [syn.upwind_1d(n, 0.1)] + [np.zeros((n, n))] * (d - 1)]
    A = ops.tt_kron_sum(terms)
    b = syn.gaussian_tt(rng, [n] * d, [1, 2, 2, 1])
    S, X, Y = _sketch_set(rng, [n] * d, 24, 25, 5)
    k = 8
    kw = dict(maxit=k, tol=1e-30, q=k, round_tol=1e-14, fixed_iterations=k, final_tol=1e-14)
    x1, i1 = solvers.tt_sgmres(A, b, S, X, Y, ls="pinv", **kw)
    x2, i2 = solvers.tt_sgmres(A, b, S, X, Y, ls="whiten", **kw)
    assert np.allclose(i1["sketched_residuals"], i2["sketched_residuals"], rtol=1e-6)
    assert np.linalg.norm(tt.full(x1) - tt.full(x2)) <= 1e-7 * np.linalg.norm(tt.full(x1))


def test_whitening_with_identity_sketch_is_gmres():
    # S = I (s = N): the whitened problem is textbook GMRES's Hessenberg problem
    n, d = 4, 3
    N = n ** d
    rng = np.random.default_rng(26)
    terms = [[syn.laplacian_1d(n)] * d, [syn.upwind_1d(n, 0.3)] + [np.zeros((n, n))] * (d - 1)]
    A = ops.tt_kron_sum(terms)
    b = syn.gaussian_tt(rng, [n] * d, [1, 2, 2, 1])
    # a Khatri-Rao factorization of the identity: row j picks the multi-index of j
    S = []
    for k in range(d):
        Sk = np.zeros((N, n))
        for j in range(N):
            Sk[j, (j // n ** (d - 1 - k)) % n] = 1.0
        S.append(Sk)
    assert np.allclose(sk.kr_dense(S), np.eye(N))
    _, X, Y = _sketch_set(rng, [n] * d, 4, 16, 4)
    k = 6
    x, info = solvers.tt_sgmres(A, b, S, X, Y, maxit=k, tol=1e-30, q=k, round_tol=1e-14, fixed_iterations=k,
                                final_tol=1e-14, ls="whiten")
    Ad = ops.dense_kron_sum(terms)
    bf = tt.full(b).reshape(-1)
    K = np.array([np.linalg.matrix_power(Ad, j) @ bf for j in range(k)]).T
    Qk, _ = np.linalg.qr(K)
    c = np.linalg.lstsq(Ad @ Qk, bf, rcond=None)[0]
    res = np.linalg.norm(bf - Ad @ Qk @ c) / np.linalg.norm(bf)
    assert abs(info["sketched_residuals"][-1] - res) <= 1e-7 * res


def test_markov_operator_against_kronecker_products():
    d, n = 3, 4
    w = syn.markov_chain(d, n, s=20, cap=16)
    At = ops.tt_markov(w["Q"], w["J"], w["P"], w["rate"])
    assert [c.shape[0] for c in At] == [1, 4, 4] and At[-1].shape[3] == 1
    Ad = ops.dense_markov(w["Q"], w["J"], w["P"], w["rate"])
    assert np.allclose(ops.dense_from_tt_matrix(At), Ad, rtol=1e-14, atol=1e-14)
    # an explicit build of one synchronization term: both systems leave state
    # n-2 for n-1 together, and D puts the matching rate on the diagonal
    N = n ** d
    idx = lambda t: int(np.ravel_multi_index(t, (n,) * d))
    i0 = idx((n - 2, n - 2, 1))
    assert Ad[i0, idx((n - 1, n - 1, 1))] == pytest.approx(w["rate"])
    diag_expect = sum(w["Q"][k][t, t] for k, t in enumerate((n - 2, n - 2, 1))) - w["rate"]
    assert Ad[i0, i0] == pytest.approx(diag_expect)
    # -A is a nonsingular M-matrix: nonpositive off-diagonal, row sums >= 0
    M = -Ad
    assert np.all(M - np.diag(np.diag(M)) <= 1e-15)
    assert np.all(M.sum(axis=1) >= -1e-12)
    assert np.linalg.matrix_rank(M) == N


def test_preconditioned_markov_solve_matches_dense():
    d, n, tol = 3, 8, 1e-6
    w = syn.markov_chain(d, n, s=40, cap=64)
    At = ops.tt_markov(w["Q"], w["J"], w["P"], w["rate"])
    # P^{-1} ~ Q^{-1} = -((+)_k (-Q_k))^{-1}: the exponential sum of the
    # positive-spectrum Kronecker sum with negated weights
    mats = [-Qk for Qk in w["Q"]]
    ev = [np.linalg.eigvals(M).real for M in mats]
    a, be = pc.expsum_coefficients(sum(e.min() for e in ev), sum(e.max() for e in ev), 1e-2)
    E = pc.mode_exponentials(be, mats)
    x, info = solvers.tt_sgmres(At, w["b"], w["S"], w["X"], w["Y"], maxit=30, tol=tol, q=1, round_tol=1e-9,
                                final_tol=1e-10, precond=(-a, E))
    assert info["true_residual"] <= tol
    Ad = ops.dense_markov(w["Q"], w["J"], w["P"], w["rate"])
    xd = np.linalg.solve(Ad, np.ones(n ** d))
    assert np.linalg.norm(tt.full(x).reshape(-1) - xd) <= 1e-4 * np.linalg.norm(xd)
