"""Pins of oracle/sketch.py: Khatri-Rao sketch against the explicit s x N matrix
and the embedding property in expectation; STTA sketches against explicitly
formed interface matrices of the DRMs; exact recovery, linearity, scale
invariance."""
import numpy as np
import pytest

import synthetic as syn
from oracle import sketch as sk
from oracle import tt


def _rand(seed, ns, ranks):
    return syn.gaussian_tt(np.random.default_rng(seed), ns, ranks)


def test_kr_sketch_against_explicit_matrix():
    ns = [3, 4, 2, 3]
    x = _rand(0, ns, [1, 2, 3, 2, 1])
    S = syn.kr_factors(np.random.default_rng(1), 7, ns)
    Sd = sk.kr_dense(S)
    # row j of the explicit matrix is the Kronecker product of the factor rows
    j = 4
    row = np.einsum('a,b,c,d->abcd', *[Sk[j] for Sk in S]).reshape(-1)
    assert np.array_equal(Sd[j], row)
    assert np.allclose(sk.kr_sketch(S, x), Sd @ tt.full(x).reshape(-1), rtol=1e-13, atol=1e-14)


def test_kr_sketch_preserves_norm_in_expectation():
    ns = [4, 4, 4]
    x = _rand(2, ns, [1, 2, 2, 1])
    nx2 = tt.norm(x) ** 2
    rng = np.random.default_rng(3)
    vals = [np.sum(sk.kr_sketch(syn.kr_factors(rng, 50, ns), x) ** 2) for _ in range(400)]
    assert abs(np.mean(vals) / nx2 - 1.0) < 0.1


def _left_interface(Y, b):
    """Y_{<=b} as a dense (n_1..n_b) x rho_b matrix."""
    M = Y[0][0]
    for c in Y[1:b]:
        M = np.tensordot(M, c, axes=([M.ndim - 1], [0]))
    return M.reshape(-1, M.shape[-1])


def _right_interface(X, b, d):
    """X_{>b} as a dense (n_{b+1}..n_d) x rX_b matrix (X holds modes 1..d-1)."""
    cores = X[b - 1:]
    M = cores[0]
    for c in cores[1:]:
        M = np.tensordot(M, c, axes=([M.ndim - 1], [0]))
    M = M[..., 0]
    return M.reshape(M.shape[0], -1).T


def test_stta_sketches_against_interface_matrices():
    ns = [3, 4, 3, 4]
    d = 4
    x = _rand(4, ns, [1, 3, 4, 2, 1])
    rng = np.random.default_rng(5)
    rx, rho = syn.stta_ranks(ns, 3, 2)
    X = syn.tt_drm(rng, ns, rx, 1, d)
    Y = syn.tt_drm(rng, ns, rho, 0, d - 1)
    Psi, Om = sk.stta_sketch(x, X, Y)
    F = tt.full(x)
    for b in range(1, d):
        T = F.reshape(int(np.prod(ns[:b])), -1)
        expect = _left_interface(Y, b).T @ T @ _right_interface(X, b, d)
        assert np.allclose(Om[b - 1], expect, rtol=1e-12, atol=1e-14)
    for mu in range(d):
        T = F.reshape(int(np.prod(ns[:mu + 1])), -1)
        left = np.eye(1) if mu == 0 else _left_interface(Y, mu)
        K = np.kron(left, np.eye(ns[mu]))
        right = np.ones((1, 1)) if mu == d - 1 else _right_interface(X, mu + 1, d)
        expect = (K.T @ T @ right).reshape(Psi[mu].shape)
        assert np.allclose(Psi[mu], expect, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("ranks", [[1, 3, 3, 3, 3, 1], [1, 1, 1, 1, 1, 1], [1, 6, 4, 2, 6, 1]])
def test_stta_exact_recovery_when_target_ranks_suffice(ranks):
    ns = [6] * 5
    x = _rand(6, ns, ranks)
    rng = np.random.default_rng(7)
    rx, rho = syn.stta_ranks(ns, 6, 3)
    X = syn.tt_drm(rng, ns, rx, 1, 5)
    Y = syn.tt_drm(rng, ns, rho, 0, 4)
    y = sk.stta_recover(*sk.stta_sketch(x, X, Y))
    assert tt.norm(tt.add(y, x, 1.0, -1.0)) <= 1e-11 * tt.norm(x)


def test_stta_linearity_and_scale_invariance():
    ns = [5] * 4
    x = _rand(8, ns, [1, 2, 3, 2, 1])
    z = _rand(9, ns, [1, 3, 2, 3, 1])
    rng = np.random.default_rng(10)
    rx, rho = syn.stta_ranks(ns, 6, 4)
    X = syn.tt_drm(rng, ns, rx, 1, 4)
    Y = syn.tt_drm(rng, ns, rho, 0, 3)
    a, b = 0.7, -1.3
    lhs = sk.stta_sketch(tt.add(x, z, a, b), X, Y)
    rhs = sk.lin_comb_sketches([a, b], [sk.stta_sketch(x, X, Y), sk.stta_sketch(z, X, Y)])
    for u, v in zip(lhs[0] + lhs[1], rhs[0] + rhs[1]):
        assert np.allclose(u, v, rtol=1e-12, atol=1e-14)
    y1 = sk.stta_recover(*sk.stta_sketch(x, X, Y))
    y2 = sk.stta_recover(*sk.stta_sketch(x, [3.0 * c for c in X], [0.25 * c for c in Y]))
    assert tt.norm(tt.add(y1, y2, 1.0, -1.0)) <= 1e-12 * tt.norm(x)


def test_round_rand_close_to_optimal_truncation():
    ns = [6] * 5
    rng = np.random.default_rng(11)
    # rank-12 tensor with geometrically decaying weights, rounded to target rank 6
    acc = None
    for j in range(12):
        t = tt.scale(syn.gaussian_tt(rng, ns, [1] * 6), 0.4 ** j)
        acc = t if acc is None else tt.add(acc, t)
    rx, rho = syn.stta_ranks(ns, 6, 6)
    X = syn.tt_drm(rng, ns, rx, 1, 5)
    Y = syn.tt_drm(rng, ns, rho, 0, 4)
    y = sk.round_rand(acc, X, Y, 0.0, 6)
    z = tt.round_svd(acc, 0.0, 6)
    e_rand = tt.norm(tt.add(y, acc, 1.0, -1.0))
    e_svd = tt.norm(tt.add(z, acc, 1.0, -1.0))
    assert e_svd <= e_rand * (1 + 1e-8)
    assert e_rand <= 100 * e_svd
    assert max(tt.ranks(y)) <= 6
