"""FP64 CPU oracle for randomized sketched TT-GMRES (Bucci, Palitta, Robol).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link anything in this package: only `tests/`, `__graft_entry__.smoke()` and the
CPU-baseline leg of `bench.py` use it.  It shares no code with the HIP path;
the only common input is the seeded generator module `synthetic`.

Everything is plain numpy/LAPACK in float64, written for readability:
  tt.py          TT format, matvec, inner products, sums, TT-SVD rounding (Sec. 2.2)
  operators.py   TT-matrix form of Kronecker-sum operators (Sec. 2.2, Sec. 5.1)
                 and of the synchronized Markov chain (Sec. 5.1.2)
  sketch.py      Khatri-Rao sketch (Sec. 3.1), Gaussian TT-DRM and STTA (Sec. 3.3)
  solvers.py     sGMRES (Alg. 1), TT-GMRES (Alg. 2), TT-sGMRES vanilla (Alg. 3)
                 and enhanced (Alg. 4), plus a deterministic twin of Alg. 4;
                 TT-sPGMRES (Alg. 5) and the whitened least squares (Sec. 3.4)
  precond.py     exponential-sum right preconditioner (Sec. 4.1)
  closed_form.py exact / exponential-sum solutions of Kronecker-sum systems
  dense.py       brute-force dense references for tiny sizes

Parity status per function is listed in each module header.
"""
