"""Pins of oracle/tt.py and oracle/operators.py against definitions that do not
go through the code under test: dense tensors, explicit Kronecker products and
numpy's SVD of unfoldings."""
import numpy as np
import pytest

import synthetic as syn
from oracle import operators as ops
from oracle import tt


def _rand(seed, ns, ranks):
    return syn.gaussian_tt(np.random.default_rng(seed), ns, ranks)


def test_full_matches_entries_and_rank1_outer_product():
    ns = [3, 4, 2, 5]
    x = _rand(0, ns, [1, 2, 3, 2, 1])
    F = tt.full(x)
    assert F.shape == tuple(ns)
    rng = np.random.default_rng(1)
    for _ in range(20):
        idx = tuple(int(rng.integers(n)) for n in ns)
        assert abs(F[idx] - tt.entry(x, idx)) < 1e-14
    vecs = [rng.standard_normal(n) for n in ns]
    r1 = [v.reshape(1, -1, 1) for v in vecs]
    outer = np.einsum('i,j,k,l->ijkl', *vecs)
    assert np.allclose(tt.full(r1), outer, rtol=0, atol=1e-15)


def test_kron_sum_dense_against_explicit_kron():
    rng = np.random.default_rng(2)
    A, B, C = (rng.standard_normal((k, k)) for k in (2, 3, 4))
    I2, I3, I4 = np.eye(2), np.eye(3), np.eye(4)
    expect = np.kron(np.kron(A, I3), I4) + np.kron(np.kron(I2, B), I4) + np.kron(np.kron(I2, I3), C)
    got = ops.dense_kron_sum([[A, B, C]])
    assert np.array_equal(got, expect)


@pytest.mark.parametrize("kind", ["laplace", "convdiff", "potential"])
def test_tt_matrix_equals_dense_operator(kind):
    n, d = 4, 3
    L = syn.laplacian_1d(n)
    if kind == "laplace":
        terms = [[L] * d]
    elif kind == "convdiff":
        terms = [[L] * d, [syn.upwind_1d(n, 0.1)] + [np.zeros((n, n))] * (d - 1)]
    else:
        terms = [[L] * d, [syn.potential_1d(n)] * d]
    A = ops.tt_kron_sum(terms)
    assert [D.shape[0] for D in A] + [A[-1].shape[3]] == [1] + [len(terms) + 1] * (d - 1) + [1]
    assert np.allclose(ops.dense_from_tt_matrix(A), ops.dense_kron_sum(terms), rtol=0, atol=1e-11)


def test_matvec_against_dense_and_rank_product():
    n, d = 4, 4
    terms = [[syn.laplacian_1d(n)] * d, [syn.potential_1d(n)] * d]
    A = ops.tt_kron_sum(terms)
    x = _rand(3, [n] * d, [1, 2, 3, 2, 1])
    y = tt.matvec(A, x)
    assert tt.ranks(y) == [1, 6, 9, 6, 1]
    expect = ops.dense_kron_sum(terms) @ tt.full(x).reshape(-1)
    assert np.allclose(tt.full(y).reshape(-1), expect, rtol=1e-13, atol=1e-12)
    yT = tt.matvec(tt.transpose_op(A), x)
    expectT = ops.dense_kron_sum(terms).T @ tt.full(x).reshape(-1)
    assert np.allclose(tt.full(yT).reshape(-1), expectT, rtol=1e-13, atol=1e-12)


def test_dot_norm_add_scale_against_full():
    ns = [3, 5, 4]
    x = _rand(4, ns, [1, 3, 2, 1])
    y = _rand(5, ns, [1, 2, 4, 1])
    Fx, Fy = tt.full(x), tt.full(y)
    assert abs(tt.dot(x, y) - np.sum(Fx * Fy)) < 1e-14
    assert abs(tt.norm(x) - np.linalg.norm(Fx)) < 1e-14
    assert np.allclose(tt.full(tt.add(x, y, 2.0, -3.0)), 2 * Fx - 3 * Fy, atol=1e-14)
    assert np.allclose(tt.full(tt.scale(x, -0.5)), -0.5 * Fx, atol=1e-15)
    z = tt.lin_comb([1.0, 2.0, -1.0], [x, y, x])
    assert np.allclose(tt.full(z), 2 * Fy, atol=1e-14)


def test_round_svd_exact_recovery_of_minimal_rank_tt():
    ns = [4, 5, 6, 3]
    x = _rand(6, ns, [1, 3, 4, 3, 1])
    padded = tt.add(x, x, 0.5, 0.5)                   # same tensor, ranks doubled
    r = tt.round_svd(padded, 0.0)
    F = tt.full(x)
    assert np.linalg.norm(tt.full(r) - F) <= 1e-13 * np.linalg.norm(F)
    # minimal ranks = matrix ranks of the unfoldings
    expect = [1] + [np.linalg.matrix_rank(F.reshape(int(np.prod(ns[:b])), -1)) for b in range(1, 4)] + [1]
    r2 = tt.round_svd(padded, 1e-12)
    assert tt.ranks(r2) == expect


def test_round_svd_error_bound_and_cap():
    rng = np.random.default_rng(7)
    ns = [5, 6, 5, 6]
    F = rng.standard_normal(ns)
    for mode in range(4):
        F = np.moveaxis(np.tensordot(np.diag(0.5 ** np.arange(ns[mode])), F, axes=([1], [mode])), 0, mode)
    x = tt.from_full(F)
    for tol in [1e-1, 1e-3, 1e-6]:
        r = tt.round_svd(x, tol)
        assert np.linalg.norm(tt.full(r) - F) <= tol * np.linalg.norm(F) * (1 + 1e-10)
        # the first bond is decided by the singular values of the first unfolding
        s = np.linalg.svd(F.reshape(ns[0], -1), compute_uv=False)
        delta = tol * np.linalg.norm(F) / np.sqrt(3)
        k = next((j for j in range(len(s)) if np.sqrt(np.sum(s[j:] ** 2)) <= delta), len(s))
        assert tt.ranks(r)[1] == max(k, 1)
    capped = tt.round_svd(x, 0.0, maxrank=2)
    assert max(tt.ranks(capped)) <= 2
