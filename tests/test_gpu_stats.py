"""GPU tests of the measurement aids: the per-class launch statistics (a
class's busy time, the union of its launches' intervals, never exceeds the sum
of their durations and equals it when every launch ran on one stream) and the
solver's single-stream mode (same results bit for bit)."""
import numpy as np
import pytest
import torch

import synthetic as syn
from oracle import operators as oops

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _ttsg():
    from paper_2409_09471_amd import ttsg
    return ttsg


def test_single_stream_busy_equals_sum():
    ttsg = _ttsg()
    n, d, s = 37, 6, 300
    rng = np.random.default_rng(11)
    x = syn.gaussian_tt(rng, [n] * d, [1, 9, 17, 23, 17, 9, 1])
    S = syn.kr_factors(rng, s, [n] * d)
    xs, Ss = ttsg.to_device(x, DEV), ttsg.to_device(S, DEV)
    ttsg.kr_sketch(Ss, xs)
    ttsg.stats_enable(True)
    try:
        for _ in range(3):
            ttsg.kr_sketch(Ss, xs)
        st = ttsg.stats_read()
    finally:
        ttsg.stats_enable(False)
    v = st["contract_f64"]
    assert v["launches"] > 0 and v["flops"] > 0
    assert 0 < v["busy"] <= v["seconds"] * (1 + 1e-9)
    # launches on one stream do not overlap (ticks of the device clock aside)
    assert v["busy"] >= 0.98 * v["seconds"]


def test_multi_stream_solve_busy_is_a_union():
    """A preconditioned solve runs independent work on several streams; its
    busy times may fall below the summed durations but never above them, and
    never below the summed time divided by the number of streams it uses."""
    ttsg = _ttsg()
    n, d = 16, 4
    w = syn.laplace_plain(d, n, b_rank=2, cap=24, s=120, q=1, maxit=20, round_tol=1e-8)
    A = oops.tt_kron_sum(w.terms)
    L = w.terms[0][0]
    ev = np.linalg.eigvalsh(L)
    alpha, beta = ttsg.expsum(d * ev.min(), d * ev.max(), 0.1)
    pre = ttsg.Preconditioner(list(alpha), list(beta), ttsg.to_device([L] * d, DEV))
    args = [ttsg.to_device(A, DEV), ttsg.to_device(w.b, DEV), ttsg.to_device(w.S, DEV), ttsg.to_device(w.X, DEV),
            ttsg.to_device(w.Y, DEV), w.rx, w.rho]
    kw = dict(maxit=w.maxit, tol=w.tol, q=w.q, round_tol=w.round_tol, maxrank=w.cap, stop_safety=w.stop_safety,
              precond=pre)
    ttsg.sgmres_solve(*args, **kw)
    ttsg.stats_enable(True)
    try:
        ttsg.sgmres_solve(*args, **kw)
        st = ttsg.stats_read()
    finally:
        ttsg.stats_enable(False)
    assert st, "no launch was recorded"
    for name, v in st.items():
        assert v["busy"] <= v["seconds"] * (1 + 1e-9), name
        assert v["busy"] >= v["seconds"] / 4 * (1 - 1e-9), name


def test_single_stream_solve_is_bit_identical():
    """The single-stream mode (every launch on the caller's stream, used for
    per-launch measurement) changes only where launches run, not what they
    compute: the same iterations, residuals and solution bit for bit."""
    ttsg = _ttsg()
    n, d = 16, 4
    w = syn.laplace_plain(d, n, b_rank=2, cap=24, s=120, q=1, maxit=20, round_tol=1e-8)
    A = oops.tt_kron_sum(w.terms)
    L = w.terms[0][0]
    ev = np.linalg.eigvalsh(L)
    alpha, beta = ttsg.expsum(d * ev.min(), d * ev.max(), 0.1)
    pre = ttsg.Preconditioner(list(alpha), list(beta), ttsg.to_device([L] * d, DEV))
    args = [ttsg.to_device(A, DEV), ttsg.to_device(w.b, DEV), ttsg.to_device(w.S, DEV), ttsg.to_device(w.X, DEV),
            ttsg.to_device(w.Y, DEV), w.rx, w.rho]
    kw = dict(maxit=w.maxit, tol=w.tol, q=w.q, round_tol=w.round_tol, maxrank=w.cap, stop_safety=w.stop_safety,
              precond=pre)
    multi = ttsg.sgmres_solve(*args, **kw)
    one = ttsg.sgmres_solve(*args, single_stream=True, **kw)
    assert one.status == multi.status == ttsg.OK
    assert one.iterations == multi.iterations
    assert one.true_residual == multi.true_residual and one.true_residual <= 1e-6
    assert one.sketched_history == multi.sketched_history
    for a, b in zip(one.x, multi.x):
        assert torch.equal(a, b)
