"""GPU parity of the comparison methods of Sec. 5.2: TT-GMRES (Alg. 2, the
deterministic baseline) and vanilla TT-sGMRES (Alg. 3, whose final solution is
formed by sequential rounded sums), against the FP64 oracle on the same inputs,
the DST closed form and dense LU, and the accuracy loss of Sec. 5.2.1 on the
GPU itself."""
import numpy as np
import pytest

import synthetic as syn
from oracle import closed_form as cf
from oracle import dense
from oracle import operators as oops
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


def dev(arrs):
    return ttsg.to_device(arrs, DEV)


def tt_rel(x, y):
    return ott.norm(ott.add(x, y, 1.0, -1.0)) / ott.norm(y)


def test_tt_gmres_laplacian_matches_oracle_and_dst():
    d, n, tol = 4, 8, 1e-6
    rng = np.random.default_rng(11)
    b = syn.gaussian_tt(rng, [n] * d, [1, 2, 2, 2, 1])
    A = oops.tt_kron_sum([[syn.laplacian_1d(n)] * d])
    print("tt_gmres laplace d=4 n=8", flush=True)
    r = ttsg.tt_gmres(dev(A), dev(b), maxit=80, tol=tol)
    xo, io = osol.tt_gmres(A, b, maxit=80, tol=tol)
    assert r.status == ttsg.OK
    # the relaxed roundings keep the same ranks, so the Arnoldi residuals agree
    m = min(8, len(io["residuals"]), len(r.sketched_history))
    assert np.allclose(r.sketched_history[:m], io["residuals"][:m], rtol=1e-6), (r.sketched_history[:m],
                                                                                io["residuals"][:m])
    assert abs(r.iterations - io["iterations"]) <= 1
    x = host(r.x)
    tr = osol.true_residual(A, b, x)
    assert abs(tr - r.true_residual) <= 1e-8 * max(tr, 1e-300) + 1e-15
    assert tr <= 3 * tol
    xe = cf.laplace_solve_full(ott.full(b))
    kappa = cf.laplace_eigs(n).max() / cf.laplace_eigs(n).min()
    assert np.linalg.norm(ott.full(x) - xe) <= kappa * 3 * tol * np.linalg.norm(xe)
    assert tt_rel(x, xo) <= kappa * 3 * tol


def test_tt_gmres_convdiff_matches_lu():
    d, n, tol = 3, 7, 1e-7
    rng = np.random.default_rng(12)
    terms = [[syn.convdiff_1d(n, K=1.0, w=3.0)] * d]
    b = syn.gaussian_tt(rng, [n] * d, [1, 2, 2, 1])
    A = oops.tt_kron_sum(terms)
    print("tt_gmres convection-diffusion d=3 n=7", flush=True)
    r = ttsg.tt_gmres(dev(A), dev(b), maxit=60, tol=tol)
    assert r.status == ttsg.OK
    x = host(r.x)
    xd = dense.solve_dense(terms, ott.full(b))
    Ad = oops.dense_kron_sum(terms)
    res = np.linalg.norm(Ad @ ott.full(x).reshape(-1) - ott.full(b).reshape(-1)) / ott.norm(b)
    assert res <= 3 * tol
    assert np.linalg.norm(ott.full(x) - xd) <= np.linalg.cond(Ad) * 3 * tol * np.linalg.norm(xd)


def test_tt_gmres_rank_cap_and_budget():
    """A rank cap below what the tolerance needs stalls the iteration: the
    budget runs out (NOT_CONVERGED) and every basis rank respects the cap."""
    d, n = 4, 8
    rng = np.random.default_rng(14)
    b = syn.gaussian_tt(rng, [n] * d, [1, 3, 3, 3, 1])
    A = oops.tt_kron_sum([[syn.laplacian_1d(n)] * d])
    r = ttsg.tt_gmres(dev(A), dev(b), maxit=12, tol=1e-10, maxrank=4)
    assert r.status == ttsg.NOT_CONVERGED and r.iterations == 12
    assert max(r.rank_history) <= 4 and max(ttsg.ranks_of(r.x)) <= 4


def _sgmres(A, b, S, X, Y, rx, rho, variant, **kw):
    return ttsg.sgmres_solve(dev(A), dev(b), dev(S), dev(X), dev(Y), rx, rho, variant=variant,
                             raise_on_error=False, **kw)


def test_vanilla_matches_oracle_vanilla():
    """Alg. 3 on the GPU against the oracle's Alg. 3 (same sketches, same loop,
    sequential rounded sums at final_tol)."""
    n, d, tol = 12, 4, 1e-6
    L = syn.laplacian_1d(n)
    terms = [[L] * d, [syn.upwind_1d(n, 0.1)] + [np.zeros((n, n))] * (d - 1)]
    A = oops.tt_kron_sum(terms)
    rng = np.random.default_rng(15)
    b = syn.gaussian_tt(rng, [n] * d, [1, 2, 2, 2, 1])
    S = syn.kr_factors(rng, 120, [n] * d)
    rx, rho = syn.stta_ranks([n] * d, 64, 20)
    X = syn.tt_drm(rng, [n] * d, rx, 1, d)
    Y = syn.tt_drm(rng, [n] * d, rho, 0, d - 1)
    # 12 steps of one cycle, no stopping test: W_k is still well conditioned, so
    # the least-squares coefficients of the GPU (incremental CGS2 QR) and of the
    # oracle (lstsq) agree, and so do the sequential rounded sums built from them.
    # (Later, W_k's conditioning decides the last digits of the sketched
    # residual, the step at which a run stops, and with it the accuracy the
    # vanilla sums keep: not pinned.)
    # With the window of one vector the conditioning of W_k grows quickly: after
    # ~15 steps the two least-squares solvers' residuals part at the 1e-6 level.
    kw = dict(maxit=12, tol=1e-12, q=1, round_tol=1e-9, final_tol=1e-9, stop_safety=0.1, max_cycles=1)
    print("vanilla TT-sGMRES d=4 n=12, 12 steps", flush=True)
    r = _sgmres(A, b, S, X, Y, rx, rho, ttsg.VARIANT_VANILLA, **kw)
    xo, io = osol.tt_sgmres(A, b, S, X, Y, variant="vanilla", fixed_iterations=12, **kw)
    assert r.iterations == 12 and io["iterations"] == 12
    dev_rel = np.abs(np.array(r.sketched_history) / np.array(io["sketched_residuals"]) - 1.0)
    print("sketched residuals gpu / oracle - 1:", [f"{v:.1e}" for v in dev_rel], flush=True)
    assert np.allclose(r.sketched_history, io["sketched_residuals"], rtol=1e-6)
    x = host(r.x)
    tr, to = osol.true_residual(A, b, x), osol.true_residual(A, b, xo)
    print(f"true residual gpu {tr:.3e} oracle {to:.3e}, solutions differ by {tt_rel(x, xo):.2e}", flush=True)
    assert abs(tr - to) <= 1e-3 * to
    assert tt_rel(x, xo) < 1e-5


def test_vanilla_loses_accuracy_enhanced_does_not_on_gpu():
    """Sec. 5.2.1 on the GPU: the paper's convection-diffusion problem (K = w =
    1e-2 on [-1, 1]^4, n = 34, rank-1 source), window 1, the same iteration run
    for 20..80 steps with the two final reconstructions.  They agree early; from
    about 40 steps the sequential rounded sums (Alg. 3) stop improving while the
    sketched sum (Alg. 4) keeps falling."""
    d, n, ftol = 4, 34, 1e-4
    A1 = syn.convdiff_1d(n)
    f = syn.gauss_source_1d(n)
    b = [f.reshape(1, n, 1).copy() for _ in range(d)]
    A = oops.tt_kron_sum([[A1] * d])
    rng = np.random.default_rng(7)
    S = syn.kr_factors(rng, 160, [n] * d)
    rx, rho = syn.stta_ranks([n] * d, 64, 20)
    X = syn.tt_drm(rng, [n] * d, rx, 1, d)
    Y = syn.tt_drm(rng, [n] * d, rho, 0, d - 1)
    enh, van = {}, {}
    for k in (20, 40, 60, 80):
        kw = dict(maxit=k, tol=1e-12, q=1, round_tol=1e-10, final_tol=ftol, stop_safety=0.1, max_cycles=1,
                  rcond=1e-8)
        print(f"E1 on the GPU: {k} iterations", flush=True)
        re = _sgmres(A, b, S, X, Y, rx, rho, ttsg.VARIANT_ENHANCED, **kw)
        rv = _sgmres(A, b, S, X, Y, rx, rho, ttsg.VARIANT_VANILLA, **kw)
        assert re.iterations == k and rv.iterations == k
        enh[k] = osol.true_residual(A, b, host(re.x))
        van[k] = osol.true_residual(A, b, host(rv.x))
    print("enhanced", enh, "vanilla", van, flush=True)
    assert abs(van[20] - enh[20]) <= 0.05 * enh[20], (van[20], enh[20])
    assert enh[80] < 0.5 * enh[20], enh
    for k in (40, 60, 80):
        assert van[k] > 3.0 * enh[k], (k, van[k], enh[k])
    assert van[80] > 0.5 * van[20], van
