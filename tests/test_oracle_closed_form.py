"""Pins of oracle/closed_form.py and oracle/dense.py: DST eigenpairs, exact DST
solve and exponential-sum solutions against dense LU, and the quadrature error
over the spectra of every workload operator."""
import numpy as np
import pytest

import synthetic as syn
from oracle import closed_form as cf
from oracle import dense
from oracle import operators as ops
from oracle import tt


def test_dst_diagonalizes_1d_laplacian():
    for n in [5, 16, 33]:
        V = cf.dst_matrix(n)
        L = syn.laplacian_1d(n)
        assert np.allclose(V @ V, np.eye(n), atol=1e-13)
        assert np.allclose(V @ L @ V, np.diag(cf.laplace_eigs(n)), atol=1e-9 * (n + 1) ** 2)
        assert np.allclose(np.sort(cf.laplace_eigs(n)), np.linalg.eigvalsh(L), rtol=1e-12)


def test_dst_solve_against_dense_lu():
    n, d = 5, 3
    b = np.random.default_rng(0).standard_normal((n,) * d)
    x = cf.laplace_solve_full(b)
    terms = [[syn.laplacian_1d(n)] * d]
    assert np.allclose(x, dense.solve_dense(terms, b), rtol=1e-12, atol=1e-15)
    assert np.allclose(dense.solve_kron_eig(terms, b), x, rtol=1e-11, atol=1e-15)


def _spectrum_range(terms, d):
    A = cf.mode_matrices(terms)
    lo = sum(np.linalg.eigvals(a).real.min() for a in A)
    hi = sum(np.linalg.eigvals(a).real.max() for a in A)
    return lo, hi


@pytest.mark.parametrize("which", ["c1", "c2", "c3_small", "c3_large", "c4", "c5"])
def test_exponential_sum_accuracy_over_workload_spectra(which):
    if which == "c1":
        terms, d = [[syn.laplacian_1d(16)] * 5], 5
    elif which == "c2":
        n, d = 64, 10
        terms = [[syn.laplacian_1d(n)] * d, [syn.upwind_1d(n, 0.1)] + [np.zeros((n, n))] * (d - 1)]
    elif which == "c3_small":
        terms, d = [[syn.laplacian_1d(32)] * 6], 6
    elif which == "c3_large":
        terms, d = [[syn.laplacian_1d(128)] * 12], 12
    elif which == "c4":
        terms, d = [[0.5 * syn.laplacian_1d(64)] + [2.0 * syn.laplacian_1d(64)] * 7], 8
    else:
        n, d = 128, 20
        terms = [[syn.laplacian_1d(n)] * d, [syn.potential_1d(n)] * d]
    lo, hi = _spectrum_range(terms, d)
    t, w = cf.expsum_nodes(lo, hi)
    assert cf.expsum_max_error(t, w, lo, hi) < 5e-13


def test_expsum_solution_against_dst_and_lu():
    n, d = 8, 4
    rng = np.random.default_rng(1)
    b = syn.gaussian_tt(rng, [n] * d, [1, 2, 2, 2, 1])
    terms = [[syn.laplacian_1d(n)] * d]
    sol = cf.kron_sum_solve_tt(terms, b)
    xe = cf.laplace_solve_full(tt.full(b))
    assert np.linalg.norm(cf.expsum_full(sol) - xe) <= 1e-12 * np.linalg.norm(xe)
    # non-symmetric convection-diffusion operator, against dense LU
    n, d = 6, 3
    b = syn.gaussian_tt(rng, [n] * d, [1, 2, 2, 1])
    terms = [[syn.laplacian_1d(n)] * d, [syn.upwind_1d(n, 0.1)] + [np.zeros((n, n))] * (d - 1)]
    sol = cf.kron_sum_solve_tt(terms, b)
    xd = dense.solve_dense(terms, tt.full(b))
    assert np.linalg.norm(cf.expsum_full(sol) - xd) <= 1e-12 * np.linalg.norm(xd)
    idx = (1, 2, 3)
    assert abs(cf.expsum_entry(sol, idx) - xd[idx]) <= 1e-12 * np.abs(xd).max()
    r = cf.expsum_round(sol, 1e-13)
    assert np.linalg.norm(tt.full(r) - xd) <= 1e-11 * np.linalg.norm(xd)
