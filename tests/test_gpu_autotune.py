"""GPU tests of the contraction tile variants and their autotuner.

All four tile variants sum every output in the same order (the split-K
decision does not depend on the tile), so a solve must give bit-identical
results whether the tuner ran, which variants it picked, or none was tuned."""
import numpy as np
import pytest
import torch

import synthetic as syn
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


def test_forced_variants_match_oracle(tmp_path):
    """Force each tile variant for the shape classes of a Khatri-Rao sketch (by
    tuning on it, then overwriting every entry with one variant) and compare
    with the oracle's sketch; all variants must agree bit for bit."""
    ttsg = _ttsg()
    n, d, s = 21, 4, 90
    rng = np.random.default_rng(8)
    x = syn.gaussian_tt(rng, [n] * d, [1, 7, 33, 5, 1])
    S = syn.kr_factors(rng, s, [n] * d)
    xs, Ss = ttsg.to_device(x, DEV), ttsg.to_device(S, DEV)
    ttsg.autotune_clear()
    ttsg.autotune(True)
    try:
        ttsg.kr_sketch(Ss, xs)
    finally:
        ttsg.autotune(False)
    path = tmp_path / "t.txt"
    ttsg.autotune_save(str(path))
    keys = [l.split()[:8] for l in path.read_text().splitlines() if not l.startswith("#")]
    assert keys
    ref = osk.kr_sketch(S, x)
    outs = []
    for v in range(4):
        forced = tmp_path / f"v{v}.txt"
        forced.write_text("".join(" ".join(k + [str(v)]) + "\n" for k in keys))
        ttsg.autotune_clear()
        ttsg.autotune_load(str(forced))
        w = ttsg.kr_sketch(Ss, xs).cpu().numpy()
        assert np.linalg.norm(w - ref) <= 1e-12 * np.linalg.norm(ref)
        outs.append(w)
    ttsg.autotune_clear()
    for w in outs[1:]:
        assert np.array_equal(w, outs[0])
