"""The allocation-free STTA sketch (ttsg_stta_sketch_noalloc) against the
workspace entry point ttsg_stta_sketch and the FP64 oracle.

Both entry points run the same kernels in the same order, so their outputs
must agree bit for bit; the oracle pins the float64 results (1e-12 relative,
as the other sketch parity tests).  The calls come in a row, larger input
first, so the second call runs on the static buffer the first one left
behind."""
import numpy as np
import pytest

import synthetic as syn
from oracle import operators as oops
from oracle import sketch as osk
from oracle import tt as ott

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2409_09471_amd import ttsg  # noqa: E402

DEV = "cuda:0"


def _case(d, n, xr, cap, over, with_op, seed):
    rng = np.random.default_rng(seed)
    ns = [n] * d
    x = syn.gaussian_tt(rng, ns, xr)
    rx, rho = syn.stta_ranks(ns, cap, over)
    X = syn.tt_drm(rng, ns, rx, 1, d)
    Y = syn.tt_drm(rng, ns, rho, 0, d - 1)
    A = None
    if with_op:
        L = syn.laplacian_1d(n)
        A = oops.tt_kron_sum([[L] * d, [syn.upwind_1d(n, 0.1)] + [np.zeros((n, n))] * (d - 1)])
    return x, X, Y, rx, rho, A


def _run_pair(case, precision):
    x, X, Y, rx, rho, A = case
    dv = lambda a: ttsg.to_device(a, DEV)  # noqa: E731
    xg, Xg, Yg = dv(x), dv(X), dv(Y)
    Ag = dv(A) if A is not None else None
    ref = ttsg.stta_sketch(xg, Xg, Yg, rx, rho, A=Ag, precision=precision)
    d, ns = len(x), [c.shape[1] for c in x]
    # outputs start as NaN: every entry must be written by the call
    out = ([torch.full((rho[k], ns[k], rx[k + 1]), float("nan"), dtype=torch.float64, device=DEV) for k in range(d)],
           [torch.full((rho[b], rx[b]), float("nan"), dtype=torch.float64, device=DEV) for b in range(1, d)])
    got = ttsg.stta_sketch_noalloc(xg, Xg, Yg, rx, rho, A=Ag, precision=precision, out=out)
    torch.cuda.synchronize()
    for g, r in zip(got[0] + got[1], ref[0] + ref[1]):
        assert torch.equal(g, r)
    return got


@pytest.mark.parametrize("precision", [ttsg.PREC_F64, ttsg.PREC_MIXED])
def test_noalloc_sketch_matches_workspace_entry_point(precision):
    big = _case(6, 24, [1, 5, 9, 12, 9, 5, 1], 16, 6, True, 71)
    small = _case(4, 10, [1, 3, 4, 2, 1], 8, 3, False, 72)
    tol = 1e-12 if precision == ttsg.PREC_F64 else 2e-5
    for case in (big, small):
        x, X, Y, rx, rho, A = case
        print(f"noalloc sketch d={len(x)} n={x[0].shape[1]} op={A is not None} precision={precision}", flush=True)
        got = _run_pair(case, precision)
        v = ott.matvec(A, x) if A is not None else x
        Po, Oo = osk.stta_sketch(v, X, Y)
        for g, o in zip(got[0] + got[1], Po + Oo):
            err = np.linalg.norm(g.cpu().numpy() - o) / np.linalg.norm(o)
            assert err <= tol, err


def test_noalloc_sketch_at_the_benchmark_shape():
    """d = 10, n = 64, ranks 64, rho 84, the rank-3 convection-diffusion
    operator (the sketch of A v_k in the benchmarked solve), then a smaller
    call on the same buffer."""
    big = _case(10, 64, [1] + [64] * 9 + [1], 64, 20, True, 73)
    print("noalloc sketch at d=10 n=64 ranks 64", flush=True)
    _run_pair(big, ttsg.PREC_F64)
    small = _case(5, 12, [1, 4, 6, 6, 4, 1], 10, 4, True, 74)
    print("noalloc sketch at d=5 n=12", flush=True)
    _run_pair(small, ttsg.PREC_F64)
