"""GPU parity of the HIP path against the FP64 oracle on the same seeded inputs.

Every test calls the library through the C ABI (ctypes binding) and compares
tensors (not cores: TT cores have gauge freedom and SVD signs are arbitrary).
FP64 results must agree to ~1e-12 relative; FP32 contractions to ~1e-5."""
import numpy as np
import pytest

import synthetic as syn
from oracle import closed_form as cf
from oracle import operators as oops
from oracle import sketch as osk
from oracle import solvers as osol
from oracle import tt as ott

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2409_09471_amd import ttsg  # noqa: E402

DEV = "cuda:0"


def host(cores):
    return [c.detach().cpu().numpy() for c in cores]


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


def tt_rel(x, y):
    """||x - y|| / ||y|| for two TTs, through the oracle's TT arithmetic."""
    return ott.norm(ott.add(x, y, 1.0, -1.0)) / ott.norm(y)


def _op(kind, n, d):
    L = syn.laplacian_1d(n)
    if kind == "laplace":
        return [[L] * d]
    if kind == "convdiff":
        return [[L] * d, [syn.upwind_1d(n, 0.1)] + [np.zeros((n, n))] * (d - 1)]
    return [[L] * d, [syn.potential_1d(n)] * d]


@pytest.mark.parametrize("kind,n,d,ranks", [
    ("laplace", 5, 3, [1, 3, 2, 1]),
    ("convdiff", 17, 4, [1, 7, 33, 5, 1]),        # several tiles and ragged tails
    ("potential", 70, 3, [1, 65, 3, 1]),
])
@pytest.mark.parametrize("transpose", [False, True])
def test_matvec(kind, n, d, ranks, transpose):
    terms = _op(kind, n, d)
    A = oops.tt_kron_sum(terms)
    x = syn.gaussian_tt(np.random.default_rng(1), [n] * d, ranks)
    y = ttsg.matvec(ttsg.to_device(A, DEV), ttsg.to_device(x, DEV), transpose=transpose)
    ref = ott.matvec(ott.transpose_op(A) if transpose else A, x)
    assert ttsg.ranks_of(y) == ott.ranks(ref)
    for g, o in zip(host(y), ref):
        assert rel(g, o) < 1e-13


@pytest.mark.parametrize("with_op", [False, True])
# BF16 rounds every operand of every stage to 8 significant bits (unit
# roundoff 2^-8); a chain of d stages then errs by a few times d * 2^-8
# norm-wise, far above FP32's 2e-5 and far below a wrong result's O(1).
@pytest.mark.parametrize("precision,tol", [(ttsg.PREC_F64, 1e-12), (ttsg.PREC_MIXED, 2e-5), (ttsg.PREC_BF16, 3e-2)])
def test_kr_sketch(with_op, precision, tol):
    n, d, s = 19, 4, 70
    terms = _op("convdiff", n, d)
    A = oops.tt_kron_sum(terms)
    rng = np.random.default_rng(2)
    x = syn.gaussian_tt(rng, [n] * d, [1, 5, 9, 4, 1])
    S = syn.kr_factors(rng, s, [n] * d)
    w = ttsg.kr_sketch(ttsg.to_device(S, DEV), ttsg.to_device(x, DEV),
                       A=ttsg.to_device(A, DEV) if with_op else None, precision=precision)
    ref = osk.kr_sketch(S, ott.matvec(A, x) if with_op else x)
    assert rel(w.cpu().numpy(), ref) < tol


@pytest.mark.parametrize("with_op", [False, True])
# BF16 rounds every operand of every stage to 8 significant bits (unit
# roundoff 2^-8); a chain of d stages then errs by a few times d * 2^-8
# norm-wise, far above FP32's 2e-5 and far below a wrong result's O(1).
@pytest.mark.parametrize("precision,tol", [(ttsg.PREC_F64, 1e-12), (ttsg.PREC_MIXED, 2e-5), (ttsg.PREC_BF16, 3e-2)])
def test_stta_sketch(with_op, precision, tol):
    n, d = 13, 5
    terms = _op("potential", n, d)
    A = oops.tt_kron_sum(terms)
    rng = np.random.default_rng(3)
    x = syn.gaussian_tt(rng, [n] * d, [1, 6, 11, 7, 3, 1])
    rx, rho = syn.stta_ranks([n] * d, 20, 7)
    X = syn.tt_drm(rng, [n] * d, rx, 1, d)
    Y = syn.tt_drm(rng, [n] * d, rho, 0, d - 1)
    Psi, Om = ttsg.stta_sketch(ttsg.to_device(x, DEV), ttsg.to_device(X, DEV), ttsg.to_device(Y, DEV), rx, rho,
                               A=ttsg.to_device(A, DEV) if with_op else None, precision=precision)
    Po, Oo = osk.stta_sketch(ott.matvec(A, x) if with_op else x, X, Y)
    for g, o in zip(host(Psi) + host(Om), Po + Oo):
        assert rel(g, o) < tol


def test_dot_and_true_residual():
    n, d = 11, 4
    terms = _op("convdiff", n, d)
    A = oops.tt_kron_sum(terms)
    rng = np.random.default_rng(4)
    x = syn.gaussian_tt(rng, [n] * d, [1, 4, 6, 3, 1])
    b = syn.gaussian_tt(rng, [n] * d, [1, 2, 2, 2, 1])
    g = ttsg.dot(ttsg.to_device(x, DEV), ttsg.to_device(b, DEV))
    assert abs(g - ott.dot(x, b)) <= 1e-13 * ott.norm(x) * ott.norm(b)
    tr = ttsg.true_residual(ttsg.to_device(A, DEV), ttsg.to_device(b, DEV), ttsg.to_device(x, DEV))
    assert abs(tr - osol.true_residual(A, b, x)) <= 1e-10 * osol.true_residual(A, b, x)


@pytest.mark.parametrize("tol,maxrank", [(0.0, 0), (1e-6, 0), (1e-2, 0), (0.0, 3)])
def test_round_svd(tol, maxrank):
    n, d = 9, 5
    rng = np.random.default_rng(5)
    acc = None
    for j in range(12):                      # decaying spectrum, rank 12 written as rank 24
        t = ott.scale(syn.gaussian_tt(rng, [n] * d, [1] * (d + 1)), 0.3 ** j)
        acc = t if acc is None else ott.add(acc, t)
    acc = ott.add(acc, acc, 0.5, 0.5)
    y = ttsg.round_svd(ttsg.to_device(acc, DEV), tol, maxrank)
    ref = ott.round_svd(acc, tol, maxrank if maxrank else None)
    yh = host(y)
    assert ttsg.ranks_of(y) == ott.ranks(ref)
    assert tt_rel(yh, ref) < 1e-10 + 1e-3 * tol
    if maxrank == 0:
        assert tt_rel(yh, acc) <= max(tol, 1e-13) * (1 + 1e-6)


@pytest.mark.parametrize("ranks,cap,tol", [([1, 3, 3, 3, 3, 1], 6, 0.0), ([1, 6, 9, 8, 5, 1], 6, 1e-8),
                                           ([1, 2, 1, 2, 1, 1], 12, 1e-10)])
def test_round_rand(ranks, cap, tol):
    n, d = 7, 5
    rng = np.random.default_rng(6)
    x = syn.gaussian_tt(rng, [n] * d, ranks)
    rx, rho = syn.stta_ranks([n] * d, cap, 5)
    X = syn.tt_drm(rng, [n] * d, rx, 1, d)
    Y = syn.tt_drm(rng, [n] * d, rho, 0, d - 1)
    y = ttsg.round_rand(ttsg.to_device(x, DEV), ttsg.to_device(X, DEV), ttsg.to_device(Y, DEV), rx, rho, tol)
    ref = osk.round_rand(x, X, Y, tol)
    assert tt_rel(host(y), ref) < 1e-9
    if max(ranks) <= cap:
        assert tt_rel(host(y), x) < 1e-9      # exact recovery at sufficient target ranks


def _solve(w, precision=ttsg.PREC_F64, **kw):
    A = ttsg.kron_sum_operator(w.terms, DEV)
    args = dict(maxit=w.maxit, tol=w.tol, q=w.q, round_tol=w.round_tol, restart=w.restart,
                stop_safety=w.stop_safety, precision=precision)
    args.update(kw)
    return ttsg.sgmres_solve(A, ttsg.to_device(w.b, DEV), ttsg.to_device(w.S, DEV), ttsg.to_device(w.X, DEV),
                             ttsg.to_device(w.Y, DEV), w.rx, w.rho, **args)


def test_sgmres_small_matches_oracle_iterates():
    w = syn.laplace_plain(4, 8, config_index=9, b_rank=2, cap=64, s=40, q=1, maxit=60, tol=1e-6, round_tol=1e-8)
    res = _solve(w)
    A = oops.tt_kron_sum(w.terms)
    xo, io = osol.tt_sgmres(A, w.b, w.S, w.X, w.Y, maxit=w.maxit, tol=w.tol, q=w.q, round_tol=w.round_tol,
                            stop_safety=w.stop_safety)
    assert res.status == ttsg.OK
    assert osol.true_residual(A, w.b, host(res.x)) <= w.tol
    # same sketches, same algorithm: the sketched residual histories agree early on
    k = min(10, len(io["sketched_residuals"]), len(res.sketched_history))
    assert np.allclose(res.sketched_history[:k], io["sketched_residuals"][:k], rtol=1e-6)
    assert tt_rel(host(res.x), xo) < 1e-5


def test_c1_fp64_solution_against_dst():
    """d=5, n=16 FP64 workload: restart 20, s=40, q=2, full STTA ranks; closed-form check."""
    w = syn.config_c1()
    res = _solve(w)
    x = host(res.x)
    xe = cf.laplace_solve_full(ott.full(w.b))
    A = oops.tt_kron_sum(w.terms)
    assert res.status == ttsg.OK
    assert osol.true_residual(A, w.b, x) <= 1e-6
    tr = osol.true_residual(A, w.b, x)
    if res.true_residual_is_bound:     # the identity's rounding floor, reported as a bound
        assert tr <= res.true_residual * (1 + 1e-9)
    else:
        assert abs(res.true_residual - tr) < 1e-8
    assert np.linalg.norm(ott.full(x) - xe) <= 1e-5 * np.linalg.norm(xe)


def _decaying_tt(rng, ns, terms, rate, rank_each=1):
    acc = None
    for j in range(terms):
        t = ott.scale(syn.gaussian_tt(rng, ns, [1] + [rank_each] * (len(ns) - 1) + [1]), rate ** j)
        acc = t if acc is None else ott.add(acc, t)
    return acc


@pytest.mark.parametrize("n,terms,rank_each,tol,maxrank", [
    (64, 16, 4, 1e-7, 0),        # unfoldings 4096 x 64: three TSQR levels
    (64, 20, 3, 1e-3, 32),       # rank cap active
    (40, 9, 5, 0.0, 0),          # ragged leaves (m = 40 * 45)
])
def test_round_svd_large(n, terms, rank_each, tol, maxrank):
    d = 4
    rng = np.random.default_rng(11)
    x = _decaying_tt(rng, [n] * d, terms, 0.5, rank_each)
    y = ttsg.round_svd(ttsg.to_device(x, DEV), tol, maxrank)
    ref = ott.round_svd(x, tol, maxrank if maxrank else None)
    assert ttsg.ranks_of(y) == ott.ranks(ref)
    assert tt_rel(host(y), ref) < 1e-9 + 1e-3 * tol
    if maxrank == 0:
        assert tt_rel(host(y), x) <= max(tol, 1e-13) * (1 + 1e-6)


def test_round_rand_workload_shapes():
    """STTA rounding of a rank-192 A v to target rank 64 (rho = 84) at n = 64, d = 5."""
    n, d = 64, 5
    rng = np.random.default_rng(12)
    terms = _op("convdiff", n, d)
    A = oops.tt_kron_sum(terms)
    v = syn.gaussian_tt(rng, [n] * d, [1, 64, 64, 64, 64, 1])
    av = ott.matvec(A, v)
    rx, rho = syn.stta_ranks([n] * d, 64, 20)
    X = syn.tt_drm(rng, [n] * d, rx, 1, d)
    Y = syn.tt_drm(rng, [n] * d, rho, 0, d - 1)
    y = ttsg.round_rand(ttsg.to_device(av, DEV), ttsg.to_device(X, DEV), ttsg.to_device(Y, DEV), rx, rho, 1e-7, 64)
    ref = osk.round_rand(av, X, Y, 1e-7, 64)
    assert ttsg.ranks_of(y) == ott.ranks(ref)
    assert tt_rel(host(y), ref) < 1e-8
