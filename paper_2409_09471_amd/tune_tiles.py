"""Tile tuner: run representative solves with the contraction autotuner on and
save the resulting tile table (one line per contraction shape class) next to
the library, where bench.py and callers can load it with ttsg.autotune_load.

    python -m paper_2409_09471_amd.tune_tiles [--out PATH]

The workloads are the convection-diffusion system (d=10, n=64, ranks <= 64)
in the mixed and FP64 modes, the preconditioned potential system (d=20,
n=128, ranks <= 128) in FP64 and a few systems of the batched Laplacian
family (caps 32); every class met is timed once on its own operands.  Tile variants
never change results, so a table tuned on one workload is safe on any other.
"""
from __future__ import annotations

import argparse
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)), "tiles_gfx950.txt"))
    args = ap.parse_args()
    import numpy as np

    import synthetic as syn
    from paper_2409_09471_amd import ttsg
    dev = "cuda:0"
    ttsg.autotune_clear()
    ttsg.autotune(True)
    try:
        w = syn.config_c2()
        A = ttsg.kron_sum_operator(w.terms, dev)
        b, S, X, Y = (ttsg.to_device(v, dev) for v in (w.b, w.S, w.X, w.Y))
        for prec in (ttsg.PREC_MIXED, ttsg.PREC_F64):
            r = ttsg.sgmres_solve(A, b, S, X, Y, w.rx, w.rho, maxit=w.maxit, tol=w.tol, q=w.q, round_tol=w.round_tol,
                                  maxrank=w.cap, stop_safety=w.stop_safety, precision=prec)
            print(f"convection-diffusion precision {prec}: {r.iterations} iterations", flush=True)
        w = syn.config_c5()
        mats = w.extra["mode_matrices"]
        ev = [np.linalg.eigvalsh(M) for M in mats]        # spectrum interval of the Kronecker sum
        alpha, beta = ttsg.expsum(sum(e.min() for e in ev), sum(e.max() for e in ev), w.extra["precond_tol"])
        pre = ttsg.Preconditioner(list(alpha), list(beta), ttsg.to_device(mats, dev))
        r = ttsg.sgmres_solve(ttsg.kron_sum_operator(w.terms, dev), *(ttsg.to_device(v, dev) for v in (w.b, w.S, w.X, w.Y)),
                              w.rx, w.rho, maxit=w.maxit, tol=w.tol, q=w.q, round_tol=w.round_tol, maxrank=w.cap,
                              stop_safety=w.stop_safety, restart=w.restart, precision=ttsg.PREC_F64, precond=pre)
        print(f"preconditioned potential d=20 n=128: {r.iterations} iterations", flush=True)
        for i, (d, n, rb) in enumerate(syn.config_c3_systems(64)[:6]):
            v = syn.config_c3_system(i, d, n, rb, maxit=40)
            r = ttsg.sgmres_solve(ttsg.kron_sum_operator(v.terms, dev), ttsg.to_device(v.b, dev),
                                  ttsg.to_device(v.S, dev), ttsg.to_device(v.X, dev), ttsg.to_device(v.Y, dev),
                                  v.rx, v.rho, maxit=v.maxit, tol=v.tol, q=v.q, round_tol=v.round_tol,
                                  maxrank=v.cap, stop_safety=v.stop_safety, precision=ttsg.PREC_MIXED)
            print(f"batched-family system d={d} n={n}: {r.iterations} iterations", flush=True)
    finally:
        ttsg.autotune(False)
    n = ttsg.autotune_save(args.out)
    print(f"{n} shape classes -> {args.out}", flush=True)


if __name__ == "__main__":
    main()
