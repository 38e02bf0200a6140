"""GPU tests of the contraction tile variants and their autotuner.

All seven tile variants sum every output in the same order (the split-K
decision does not depend on the tile), so a solve must give bit-identical
results whether the tuner ran, which variants it picked, or none was tuned."""
import numpy as np
import pytest
import torch

import synthetic as syn
from oracle import operators as oops
from oracle import sketch as osk
from oracle import tt as ott

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _ttsg():
    from paper_2409_09471_amd import ttsg
    return ttsg


def _solve(ttsg, w, t, precision):
    return ttsg.sgmres_solve(t["A"], t["b"], t["S"], t["X"], t["Y"], w.rx, w.rho, maxit=w.maxit, tol=w.tol, q=w.q,
                             round_tol=w.round_tol, maxrank=w.cap, stop_safety=w.stop_safety, precision=precision)


@pytest.mark.parametrize("precision", [0, 1])
def test_tuned_solve_is_bit_identical(precision, tmp_path):
    ttsg = _ttsg()
    w = syn.laplace_plain(5, 12, b_rank=3, cap=40, s=200, q=1, maxit=120, round_tol=1e-8)
    t = dict(A=ttsg.kron_sum_operator(w.terms, DEV), b=ttsg.to_device(w.b, DEV), S=ttsg.to_device(w.S, DEV),
             X=ttsg.to_device(w.X, DEV), Y=ttsg.to_device(w.Y, DEV))
    ttsg.autotune(False)
    ttsg.autotune_clear()
    ref = _solve(ttsg, w, t, precision)
    ttsg.autotune(True)
    try:
        tuned = _solve(ttsg, w, t, precision)
    finally:
        ttsg.autotune(False)
    n = ttsg.autotune_save(str(tmp_path / "tiles.txt"))
    assert n > 0
    again = _solve(ttsg, w, t, precision)
    for r in (tuned, again):
        assert r.iterations == ref.iterations
        assert r.true_residual == ref.true_residual
        for a, b in zip(ref.x, r.x):
            assert torch.equal(a, b)
    ttsg.autotune_clear()


@pytest.mark.parametrize("with_op,precision,tol", [(False, 0, 1e-12), (True, 0, 1e-12), (True, 1, 2e-5)])
def test_forced_variants_match_oracle(tmp_path, with_op, precision, tol):
    """Force each tile variant (32 x 32 up to 128 x 128) for the shape classes
    of a Khatri-Rao sketch (by tuning on it, then overwriting every entry with
    one variant) and compare with the oracle's sketch; all variants must agree
    bit for bit.  With the operator (rank 3, so the Khatri-Rao operand is formed
    inside the contraction's staging) in FP64 and FP32."""
    ttsg = _ttsg()
    n, d, s = 21, 4, 90
    rng = np.random.default_rng(8)
    x = syn.gaussian_tt(rng, [n] * d, [1, 7, 33, 5, 1])
    S = syn.kr_factors(rng, s, [n] * d)
    terms = [[syn.laplacian_1d(n)] * d, [np.diag(rng.standard_normal(n)) for _ in range(d)]]
    xs, Ss = ttsg.to_device(x, DEV), ttsg.to_device(S, DEV)
    As = ttsg.kron_sum_operator(terms, DEV) if with_op else None
    ttsg.autotune_clear()
    ttsg.autotune(True)
    try:
        ttsg.kr_sketch(Ss, xs, A=As, precision=precision)
    finally:
        ttsg.autotune(False)
    path = tmp_path / "t.txt"
    ttsg.autotune_save(str(path))
    keys = [l.split()[:8] for l in path.read_text().splitlines() if not l.startswith("#")]
    assert keys
    ref = osk.kr_sketch(S, ott.matvec(oops.tt_kron_sum(terms), x) if with_op else x)
    outs = []
    for v in range(7):
        forced = tmp_path / f"v{v}.txt"
        forced.write_text("".join(" ".join(k + [str(v)]) + "\n" for k in keys))
        ttsg.autotune_clear()
        assert ttsg.autotune_load(str(forced)) == len(keys)
        w = ttsg.kr_sketch(Ss, xs, A=As, precision=precision).double().cpu().numpy()
        assert np.linalg.norm(w - ref) <= tol * np.linalg.norm(ref), v
        outs.append(w)
    ttsg.autotune_clear()
    for v, w in enumerate(outs[1:], 1):
        assert np.array_equal(w, outs[0]), v


def test_forced_variants_plain_contractions_agree(tmp_path):
    """Every tile variant forced on the plain contractions of an STTA sketch of
    A x (environment steps, Psi/Omega products, split-K reductions): the
    sketches must equal the oracle's and each other bit for bit."""
    ttsg = _ttsg()
    n, d = 17, 4
    rng = np.random.default_rng(9)
    x = syn.gaussian_tt(rng, [n] * d, [1, 9, 40, 6, 1])
    terms = [[syn.laplacian_1d(n)] * d, [np.diag(rng.standard_normal(n)) for _ in range(d)]]
    rx, rho = syn.stta_ranks([n] * d, 40, 20)
    X = syn.tt_drm(rng, [n] * d, rx, 1, d)
    Y = syn.tt_drm(rng, [n] * d, rho, 0, d - 1)
    xs, Xs, Ys = ttsg.to_device(x, DEV), ttsg.to_device(X, DEV), ttsg.to_device(Y, DEV)
    As = ttsg.kron_sum_operator(terms, DEV)
    ttsg.autotune_clear()
    ttsg.autotune(True)
    try:
        ttsg.stta_sketch(xs, Xs, Ys, rx, rho, A=As)
    finally:
        ttsg.autotune(False)
    path = tmp_path / "t.txt"
    ttsg.autotune_save(str(path))
    keys = [l.split()[:8] for l in path.read_text().splitlines() if not l.startswith("#")]
    assert keys
    Ax = ott.matvec(oops.tt_kron_sum(terms), x)
    Psi_o, Om_o = osk.stta_sketch(Ax, X, Y)
    outs = []
    for v in range(7):
        forced = tmp_path / f"p{v}.txt"
        forced.write_text("".join(" ".join(k + [str(v)]) + "\n" for k in keys))
        ttsg.autotune_clear()
        assert ttsg.autotune_load(str(forced)) == len(keys)
        Psi, Om = ttsg.stta_sketch(xs, Xs, Ys, rx, rho, A=As)
        Psi = [p.cpu().numpy() for p in Psi]
        Om = [o.cpu().numpy() for o in Om]
        for a, b in zip(Psi, Psi_o):
            assert np.linalg.norm(a - b.reshape(a.shape)) <= 1e-12 * np.linalg.norm(b), v
        for a, b in zip(Om, Om_o):
            assert np.linalg.norm(a - b.reshape(a.shape)) <= 1e-12 * np.linalg.norm(b), v
        outs.append(Psi + Om)
    ttsg.autotune_clear()
    for v, o in enumerate(outs[1:], 1):
        assert all(np.array_equal(a, b) for a, b in zip(o, outs[0])), v
