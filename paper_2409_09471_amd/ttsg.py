"""ctypes binding of libttsg (include/ttsg.h).

Argument marshalling only: every numerical step runs in the HIP library.
PyTorch provides device memory (float64 CUDA tensors) and the current HIP
stream.  TT cores are passed as lists of contiguous float64 device tensors of
shape (r_k, n_k, r_{k+1}); operator cores as (R_k, n_k, n_k, R_{k+1}).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libttsg.so")

PREC_F64 = 0
PREC_MIXED = 1
PREC_BF16 = 2

OK = 0
NOT_CONVERGED = 1
BREAKDOWN = 2
RANK_CAPPED = 3

ERR_ARG = -1
ERR_CAPACITY = -2
ERR_WS = -3
ERR_NONFINITE = -4
ERR_HIP = -5
ERR_DTYPE = -6

LS_PINV = 0
LS_WHITEN = 1
VARIANT_ENHANCED = 0   # Alg. 4: the cycle's solution recovered from the combined sketches
VARIANT_VANILLA = 1    # Alg. 3: sequential rounded sums of the kept basis vectors

_lib = None


class TTSGError(RuntimeError):
    def __init__(self, msg, code=0):
        super().__init__(msg)
        self.code = code


def lib():
    """Load libttsg.so; raise if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise TTSGError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
        L = ctypes.CDLL(LIB_PATH)
        L.ttsg_last_error.restype = ctypes.c_char_p
        L.ttsg_version.restype = ctypes.c_char_p
        _lib = L
    return _lib


EXPORTED = [
    "ttsg_last_error", "ttsg_version", "ttsg_matvec", "ttsg_kr_sketch", "ttsg_stta_sketch",
    "ttsg_round_rand", "ttsg_round_svd", "ttsg_sgmres_solve", "ttsg_true_residual", "ttsg_dot",
    "ttsg_sgmres_solve_batched", "ttsg_autotune", "ttsg_autotune_save", "ttsg_autotune_load", "ttsg_autotune_clear",
    "ttsg_grad_kron_sum", "ttsg_tt_axpby", "ttsg_stats_enable", "ttsg_stats_read",
    "ttsg_sgmres_solve_ex", "ttsg_sgmres_workspace_size", "ttsg_expsum", "ttsg_precond_round",
    "ttsg_kr_sketch_workspace_size", "ttsg_stta_sketch_workspace_size", "ttsg_round_rand_workspace_size",
    "ttsg_stta_sketch_noalloc", "ttsg_tt_gmres", "ttsg_tt_gmres_workspace_size",
]

STAT_CLASSES = {0: "contract_f64", 1: "contract_f32", 2: "contract_bf16", 3: "qr", 4: "svd_jacobi",
                5: "qr_redo"}


class Stats(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64 * 8), ("flops", ctypes.c_double * 8),
                ("bytes", ctypes.c_double * 8), ("seconds", ctypes.c_double * 8), ("busy", ctypes.c_double * 8)]


def autotune(on: bool = True) -> bool:
    """Start (or stop) timing the tile variants of new contraction shape classes."""
    return bool(lib().ttsg_autotune(int(on)))


def autotune_save(path: str) -> int:
    return _check(lib().ttsg_autotune_save(os.fsencode(path)), "ttsg_autotune_save")


def autotune_load(path: str) -> int:
    return _check(lib().ttsg_autotune_load(os.fsencode(path)), "ttsg_autotune_load")


def autotune_clear() -> int:
    return lib().ttsg_autotune_clear()


def stats_enable(on: bool = True) -> None:
    _check(lib().ttsg_stats_enable(int(on)), "ttsg_stats_enable")


def stats_read() -> dict:
    st = Stats()
    _check(lib().ttsg_stats_read(ctypes.byref(st)), "ttsg_stats_read")
    out = {}
    for c, name in STAT_CLASSES.items():
        if st.launches[c]:
            out[name] = dict(launches=int(st.launches[c]), flops=st.flops[c], bytes=st.bytes[c],
                             seconds=st.seconds[c], busy=st.busy[c])
    return out


class SgmresOpts(ctypes.Structure):
    _fields_ = [
        ("maxit", ctypes.c_int32), ("restart", ctypes.c_int32), ("q", ctypes.c_int32),
        ("maxrank", ctypes.c_int32), ("precision", ctypes.c_int32), ("max_cycles", ctypes.c_int32),
        ("tol", ctypes.c_double), ("round_tol", ctypes.c_double), ("final_tol", ctypes.c_double),
        ("stop_safety", ctypes.c_double), ("rcond", ctypes.c_double),
    ]


class SgmresInfo(ctypes.Structure):
    _fields_ = [
        ("iterations", ctypes.c_int32), ("cycles", ctypes.c_int32), ("max_rank", ctypes.c_int32),
        ("status", ctypes.c_int32), ("true_residual", ctypes.c_double),
        ("sketched_residual", ctypes.c_double),
        ("sketched_history", ctypes.POINTER(ctypes.c_double)),
        ("rank_history", ctypes.POINTER(ctypes.c_int32)),
        ("true_history", ctypes.POINTER(ctypes.c_double)),
        ("phase_seconds", ctypes.POINTER(ctypes.c_double)),
        ("true_residual_is_bound", ctypes.c_int32),
    ]


class SgmresExt(ctypes.Structure):
    _fields_ = [
        ("x0_r", ctypes.c_void_p), ("x0", ctypes.c_void_p),
        ("zeta", ctypes.c_int32), ("alpha", ctypes.c_void_p), ("beta", ctypes.c_void_p), ("M", ctypes.c_void_p),
        ("ls_mode", ctypes.c_int32), ("variant", ctypes.c_int32), ("single_stream", ctypes.c_int32),
    ]


PHASES = ["kr_sketch", "inner_products", "stta_sketch", "stta_recover", "tt_svd", "least_squares",
          "final_solution", "other"]


def _i32(vals) -> ctypes.Array:
    return (ctypes.c_int32 * len(vals))(*[int(v) for v in vals])


def _ptrs(tensors) -> ctypes.Array:
    for t in tensors:
        if t.dtype != torch.float64 or not t.is_contiguous() or not t.is_cuda:
            raise TTSGError("cores must be contiguous float64 CUDA tensors")
    return (ctypes.c_void_p * len(tensors))(*[t.data_ptr() for t in tensors])


def _stream() -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check(rc: int, what: str) -> int:
    if rc < 0:
        msg = lib().ttsg_last_error().decode()
        raise TTSGError(f"{what} failed ({rc}): {msg}", rc)
    return rc


def _workspace(nbytes: int, device) -> torch.Tensor:
    """Caller-owned scratch for one call (the library then allocates nothing)."""
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def ranks_of(cores: Sequence[torch.Tensor]) -> List[int]:
    return [int(c.shape[0]) for c in cores] + [int(cores[-1].shape[2])]


def sizes_of(cores: Sequence[torch.Tensor]) -> List[int]:
    return [int(c.shape[1]) for c in cores]


def op_ranks(cores: Sequence[torch.Tensor]) -> List[int]:
    return [int(c.shape[0]) for c in cores] + [int(cores[-1].shape[3])]


def to_device(arrays, device="cuda") -> List[torch.Tensor]:
    return [torch.as_tensor(a, dtype=torch.float64).contiguous().to(device) for a in arrays]


# ----------------------------------------------------------------------------
# Problem setup: Kronecker-sum operators in TT-matrix form (Sec. 2.2, Sec. 5.1)
# ----------------------------------------------------------------------------

def kron_sum_operator(terms, device="cuda") -> List[torch.Tensor]:
    """TT-matrix cores of sum_t sum_k (I x .. x terms[t][k] x .. x I).

    Bond state 0 means "nothing placed yet", state t+1 "the matrix of term t has
    been placed"; the last core folds all states into one (rank len(terms)+1)."""
    import numpy as np
    nterm = len(terms)
    d = len(terms[0])
    R = nterm + 1
    cores = []
    for k in range(d):
        n = terms[0][k].shape[0]
        eye = np.eye(n)
        left = 1 if k == 0 else R
        right = 1 if k == d - 1 else R
        D = np.zeros((left, n, n, right))
        if d == 1:
            D[0, :, :, 0] = sum(t[k] for t in terms)
        elif k == d - 1:
            D[0, :, :, 0] = sum(t[k] for t in terms)
            for t in range(nterm):
                D[t + 1, :, :, 0] = eye
        else:
            D[0, :, :, 0] = eye
            for t in range(nterm):
                D[0, :, :, t + 1] = terms[t][k]
                if k > 0:
                    D[t + 1, :, :, t + 1] = eye
        cores.append(D)
    return to_device(cores, device)


def markov_operator(Q, J, P, rate: float, device="cuda") -> List[torch.Tensor]:
    """TT-matrix cores of the synchronized Markov chain (Sec. 5.1.2):
    sum_k Q_k + rate sum_k (J_k x J_{k+1}) - rate sum_k (P_k x P_{k+1}).

    Bond states: 0 = nothing placed, 1 = a term completed, 2 = the J of a
    synchronization pair is open, 3 = its P is open (closed on the next mode)."""
    import numpy as np
    d = len(Q)
    n = Q[0].shape[0]
    eye = np.eye(n)
    cores = []
    for k in range(d):
        left = [0] if k == 0 else [0, 1, 2, 3]
        right = [1] if k == d - 1 else [0, 1, 2, 3]
        D = np.zeros((len(left), n, n, len(right)))
        blocks = {(0, 0): eye, (1, 1): eye, (0, 1): Q[k], (0, 2): rate * J, (0, 3): -rate * P,
                  (2, 1): J, (3, 1): P}
        for (a, b), blk in blocks.items():
            if a in left and b in right:
                D[left.index(a), :, :, right.index(b)] = blk
        cores.append(D)
    return to_device(cores, device)


# ----------------------------------------------------------------------------
# Entry points
# ----------------------------------------------------------------------------

def matvec(A: Sequence[torch.Tensor], x: Sequence[torch.Tensor], transpose: bool = False) -> List[torch.Tensor]:
    d = len(x)
    n, r, R = sizes_of(x), ranks_of(x), op_ranks(A)
    y = [torch.empty((r[k] * R[k], n[k], r[k + 1] * R[k + 1]), dtype=torch.float64, device=x[0].device)
         for k in range(d)]
    _check(lib().ttsg_matvec(d, _i32(n), _i32(R), _ptrs(A), _i32(r), _ptrs(x), int(transpose), _ptrs(y),
                             _stream()), "ttsg_matvec")
    return y


def kr_sketch(S: Sequence[torch.Tensor], x: Sequence[torch.Tensor], A: Optional[Sequence[torch.Tensor]] = None,
              precision: int = PREC_F64) -> torch.Tensor:
    d = len(x)
    s = int(S[0].shape[0])
    w = torch.empty(s, dtype=torch.float64, device=x[0].device)
    Rp = _i32(op_ranks(A)) if A is not None else None
    Ap = _ptrs(A) if A is not None else None
    nb = ctypes.c_size_t(0)
    _check(lib().ttsg_kr_sketch_workspace_size(d, _i32(sizes_of(x)), s, Rp, _i32(ranks_of(x)), precision,
                                               ctypes.byref(nb)), "ttsg_kr_sketch_workspace_size")
    ws = _workspace(nb.value, x[0].device)
    _check(lib().ttsg_kr_sketch(d, _i32(sizes_of(x)), s, _ptrs(S), Rp, Ap, _i32(ranks_of(x)), _ptrs(x),
                                ctypes.c_void_p(w.data_ptr()), precision, ctypes.c_void_p(ws.data_ptr()), nb,
                                _stream()), "ttsg_kr_sketch")
    return w


def stta_sketch(x, X, Y, rx, rho, A=None, precision: int = PREC_F64):
    """Psi (d cores rho_k x n_k x rx_{k+1}) and Omega (d-1 matrices rho_b x rx_b)."""
    d = len(x)
    n = sizes_of(x)
    dev = x[0].device
    Psi = [torch.empty((rho[k], n[k], rx[k + 1]), dtype=torch.float64, device=dev) for k in range(d)]
    Om = [torch.empty((rho[b], rx[b]), dtype=torch.float64, device=dev) for b in range(1, d)]
    Rp = _i32(op_ranks(A)) if A is not None else None
    Ap = _ptrs(A) if A is not None else None
    nb = ctypes.c_size_t(0)
    _check(lib().ttsg_stta_sketch_workspace_size(d, _i32(n), _i32(rho), _i32(rx), Rp, _i32(ranks_of(x)), precision,
                                                 ctypes.byref(nb)), "ttsg_stta_sketch_workspace_size")
    ws = _workspace(nb.value, dev)
    _check(lib().ttsg_stta_sketch(d, _i32(n), _i32(rho), _ptrs(Y), _i32(rx), _ptrs(X), Rp, Ap, _i32(ranks_of(x)),
                                  _ptrs(x), _ptrs(Psi), _ptrs(Om), precision, ctypes.c_void_p(ws.data_ptr()), nb,
                                  _stream()), "ttsg_stta_sketch")
    return Psi, Om


def stta_sketch_noalloc(x, X, Y, rx, rho, A=None, precision: int = PREC_F64, out=None):
    """ttsg_stta_sketch_noalloc: the sketch with the library's static scratch
    (no workspace).  `out` = (Psi, Om) lists to write into (allocated here
    when None)."""
    d = len(x)
    n = sizes_of(x)
    dev = x[0].device
    if out is None:
        Psi = [torch.empty((rho[k], n[k], rx[k + 1]), dtype=torch.float64, device=dev) for k in range(d)]
        Om = [torch.empty((rho[b], rx[b]), dtype=torch.float64, device=dev) for b in range(1, d)]
    else:
        Psi, Om = out
    Rp = _i32(op_ranks(A)) if A is not None else None
    Ap = _ptrs(A) if A is not None else None
    _check(lib().ttsg_stta_sketch_noalloc(d, _i32(n), _i32(rho), _ptrs(Y), _i32(rx), _ptrs(X), Rp, Ap,
                                          _i32(ranks_of(x)), _ptrs(x), _ptrs(Psi), _ptrs(Om), precision, _stream()),
           "ttsg_stta_sketch_noalloc")
    return Psi, Om


def _trim(cores, r):
    return [c.reshape(-1)[: r[k] * c.shape[1] * r[k + 1]].reshape(r[k], c.shape[1], r[k + 1]).clone()
            for k, c in enumerate(cores)]


def round_rand(x, X, Y, rx, rho, tol: float, maxrank: int = 0, rcond: float = 1e-12,
               precision: int = PREC_F64) -> List[torch.Tensor]:
    d = len(x)
    n = sizes_of(x)
    dev = x[0].device
    out = [torch.empty((rx[k], n[k], rx[k + 1]), dtype=torch.float64, device=dev) for k in range(d)]
    out_r = (ctypes.c_int32 * (d + 1))()
    nb = ctypes.c_size_t(0)
    _check(lib().ttsg_round_rand_workspace_size(d, _i32(n), _i32(ranks_of(x)), _i32(rho), _i32(rx), precision,
                                                ctypes.byref(nb)), "ttsg_round_rand_workspace_size")
    ws = _workspace(nb.value, dev)
    _check(lib().ttsg_round_rand(d, _i32(n), _i32(ranks_of(x)), _ptrs(x), _i32(rho), _ptrs(Y), _i32(rx), _ptrs(X),
                                 ctypes.c_double(tol), int(maxrank), ctypes.c_double(rcond), _ptrs(out), out_r,
                                 precision, ctypes.c_void_p(ws.data_ptr()), nb, _stream()), "ttsg_round_rand")
    return _trim(out, list(out_r))


def round_svd(x, tol: float, maxrank: int = 0) -> List[torch.Tensor]:
    d = len(x)
    out = [torch.empty_like(c) for c in x]
    out_r = (ctypes.c_int32 * (d + 1))()
    _check(lib().ttsg_round_svd(d, _i32(sizes_of(x)), _i32(ranks_of(x)), _ptrs(x), ctypes.c_double(tol),
                                int(maxrank), _ptrs(out), out_r, None, ctypes.c_size_t(0), _stream()),
           "ttsg_round_svd")
    return _trim(out, list(out_r))


def dot(x, y) -> float:
    out = ctypes.c_double(0.0)
    _check(lib().ttsg_dot(len(x), _i32(sizes_of(x)), _i32(ranks_of(x)), _ptrs(x), _i32(ranks_of(y)), _ptrs(y),
                          ctypes.byref(out), None, ctypes.c_size_t(0), _stream()), "ttsg_dot")
    return out.value


def grad_kron_sum(Ls, lam, x):
    """[-<lam, L_k x>]_k for mode operators L_k (n_k x n_k CUDA float64 tensors)."""
    import numpy as np
    d = len(x)
    for k, L in enumerate(Ls):
        if tuple(L.shape) != (x[k].shape[1], x[k].shape[1]):
            raise TTSGError(f"grad_kron_sum: L[{k}] has shape {tuple(L.shape)}")
    out = (ctypes.c_double * d)()
    _check(lib().ttsg_grad_kron_sum(d, _i32(sizes_of(x)), _ptrs(Ls), _i32(ranks_of(lam)), _ptrs(lam),
                                    _i32(ranks_of(x)), _ptrs(x), out, None, ctypes.c_size_t(0), _stream()),
           "ttsg_grad_kron_sum")
    return np.array([out[k] for k in range(d)])


def tt_axpby(alpha: float, x, beta: float, y) -> List[torch.Tensor]:
    """alpha x + beta y as a block TT (ranks add on the inner bonds)."""
    d = len(x)
    n = sizes_of(x)
    rx, ry = ranks_of(x), ranks_of(y)
    rz = [1] + [rx[k] + ry[k] for k in range(1, d)] + [1] if d > 1 else [1, 1]
    z = [torch.empty((rz[k], n[k], rz[k + 1]), dtype=torch.float64, device=x[0].device) for k in range(d)]
    _check(lib().ttsg_tt_axpby(d, _i32(n), ctypes.c_double(alpha), _i32(rx), _ptrs(x), ctypes.c_double(beta),
                               _i32(ry), _ptrs(y), _ptrs(z), _stream()), "ttsg_tt_axpby")
    return z


def true_residual(A, b, x) -> float:
    out = ctypes.c_double(0.0)
    _check(lib().ttsg_true_residual(len(x), _i32(sizes_of(x)), _i32(op_ranks(A)), _ptrs(A), _i32(ranks_of(b)),
                                    _ptrs(b), _i32(ranks_of(x)), _ptrs(x), ctypes.byref(out), None,
                                    ctypes.c_size_t(0), _stream()), "ttsg_true_residual")
    return out.value


@dataclass
class SolveResult:
    x: List[torch.Tensor]
    status: int
    iterations: int
    cycles: int
    true_residual: float
    sketched_residual: float
    max_rank: int
    sketched_history: List[float] = field(default_factory=list)
    rank_history: List[int] = field(default_factory=list)
    true_history: List[float] = field(default_factory=list)
    phase_seconds: dict = field(default_factory=dict)
    # the reported true residual is the rounding floor of the FP64 identity
    # (an upper bound), not a measured norm
    true_residual_is_bound: bool = False


@dataclass
class Preconditioner:
    """Exponential-sum right preconditioner P^{-1} = sum_j alpha[j] (x)_k exp(-beta[j] M[k])
    (Sec. 4.1): M are the d mode matrices (CUDA float64, n_k x n_k)."""
    alpha: Sequence[float]
    beta: Sequence[float]
    M: List[torch.Tensor]


def expsum(zmin: float, zmax: float, tol: float, max_terms: int = 1024):
    """(alpha, beta) with |z E(z) - 1| <= tol on [zmin, zmax] (ttsg_expsum)."""
    import numpy as np
    a = (ctypes.c_double * max_terms)()
    b = (ctypes.c_double * max_terms)()
    z = _check(lib().ttsg_expsum(ctypes.c_double(zmin), ctypes.c_double(zmax), ctypes.c_double(tol),
                                 int(max_terms), a, b), "ttsg_expsum")
    return np.array(a[:z]), np.array(b[:z])


def _dbl(vals) -> ctypes.Array:
    return (ctypes.c_double * len(vals))(*[float(v) for v in vals])


def precond_round(x, pre: Preconditioner, X, Y, rx, rho, tol: float, maxrank: int = 0,
                  rcond: float = 1e-12) -> List[torch.Tensor]:
    """Round(P^{-1} x) by the STTA streaming sum of the preconditioner's terms."""
    d = len(x)
    n = sizes_of(x)
    dev = x[0].device
    out = [torch.empty((rx[k], n[k], rx[k + 1]), dtype=torch.float64, device=dev) for k in range(d)]
    out_r = (ctypes.c_int32 * (d + 1))()
    _check(lib().ttsg_precond_round(d, _i32(n), len(pre.alpha), _dbl(pre.alpha), _dbl(pre.beta), _ptrs(pre.M),
                                    _i32(ranks_of(x)), _ptrs(x), _i32(rho), _ptrs(Y), _i32(rx), _ptrs(X),
                                    ctypes.c_double(tol), int(maxrank), ctypes.c_double(rcond), _ptrs(out), out_r,
                                    None, ctypes.c_size_t(0), _stream()), "ttsg_precond_round")
    return _trim(out, list(out_r))


def sgmres_workspace_size(A, b, S, rx, rho, opts: "SgmresOpts", ext: Optional["SgmresExt"] = None) -> int:
    nb = ctypes.c_size_t(0)
    _check(lib().ttsg_sgmres_workspace_size(len(b), _i32(sizes_of(b)), _i32(op_ranks(A)), _i32(ranks_of(b)),
                                            int(S[0].shape[0]), _i32(rho), _i32(rx), ctypes.byref(opts),
                                            ctypes.byref(ext) if ext is not None else None, ctypes.byref(nb)),
           "ttsg_sgmres_workspace_size")
    return nb.value


def sgmres_solve(A, b, S, X, Y, rx, rho, *, maxit: int, tol: float, q: int = 1, round_tol: float = 1e-7,
                 maxrank: int = 0, restart: int = 0, final_tol: float = 0.0, stop_safety: float = 0.1,
                 rcond: float = 1e-12, precision: int = PREC_F64, max_cycles: int = 50,
                 phase_timing: bool = False, x0: Optional[Sequence[torch.Tensor]] = None,
                 precond: Optional[Preconditioner] = None, ls: int = LS_PINV, variant: int = VARIANT_ENHANCED,
                 single_stream: bool = False, workspace: Optional[torch.Tensor] = None,
                 raise_on_error: bool = True) -> SolveResult:
    """Alg. 4 (Alg. 5 with `precond`).  The workspace is queried and allocated
    here (or passed in), so the library allocates no device memory.  With
    `single_stream` every launch goes to torch's current stream in order."""
    d = len(b)
    n = sizes_of(b)
    dev = b[0].device
    opts = SgmresOpts(maxit=maxit, restart=restart, q=q, maxrank=maxrank, precision=precision,
                      max_cycles=max_cycles, tol=tol, round_tol=round_tol, final_tol=final_tol,
                      stop_safety=stop_safety, rcond=rcond)
    keep = []
    ext = SgmresExt(ls_mode=int(ls), variant=int(variant), single_stream=int(bool(single_stream)))
    if x0 is not None:
        r0a, p0a = _i32(ranks_of(x0)), _ptrs(x0)
        keep += [r0a, p0a]
        ext.x0_r = ctypes.cast(r0a, ctypes.c_void_p)
        ext.x0 = ctypes.cast(p0a, ctypes.c_void_p)
    if precond is not None:
        aa, ba, ma = _dbl(precond.alpha), _dbl(precond.beta), _ptrs(precond.M)
        keep += [aa, ba, ma]
        ext.zeta = len(precond.alpha)
        ext.alpha = ctypes.cast(aa, ctypes.c_void_p)
        ext.beta = ctypes.cast(ba, ctypes.c_void_p)
        ext.M = ctypes.cast(ma, ctypes.c_void_p)
    if workspace is None:
        workspace = _workspace(sgmres_workspace_size(A, b, S, rx, rho, opts, ext), dev)
    sh = (ctypes.c_double * maxit)()
    rh = (ctypes.c_int32 * maxit)()
    th = (ctypes.c_double * max_cycles)()
    ph = (ctypes.c_double * 8)()
    info = SgmresInfo(sketched_history=sh, rank_history=rh, true_history=th,
                      phase_seconds=ph if phase_timing else None)
    x = [torch.zeros((rx[k], n[k], rx[k + 1]), dtype=torch.float64, device=dev) for k in range(d)]
    xr = (ctypes.c_int32 * (d + 1))()
    rc = lib().ttsg_sgmres_solve_ex(d, _i32(n), _i32(op_ranks(A)), _ptrs(A), _i32(ranks_of(b)), _ptrs(b),
                                    int(S[0].shape[0]), _ptrs(S), _i32(rho), _ptrs(Y), _i32(rx), _ptrs(X),
                                    ctypes.byref(opts), ctypes.byref(ext), _ptrs(x), xr, ctypes.byref(info),
                                    ctypes.c_void_p(workspace.data_ptr()), ctypes.c_size_t(workspace.numel()),
                                    _stream())
    if raise_on_error:
        _check(rc, "ttsg_sgmres_solve")
    elif rc < 0:
        return SolveResult(x=[], status=rc, iterations=0, cycles=0, true_residual=float("nan"),
                           sketched_residual=float("nan"), max_rank=0)
    it = info.iterations
    return SolveResult(
        x=_trim(x, list(xr)), status=rc, iterations=it, cycles=info.cycles,
        true_residual=info.true_residual, sketched_residual=info.sketched_residual, max_rank=info.max_rank,
        true_residual_is_bound=bool(info.true_residual_is_bound),
        sketched_history=[sh[i] for i in range(min(it, maxit))],
        rank_history=[rh[i] for i in range(min(it, maxit))],
        true_history=[th[i] for i in range(min(info.cycles, max_cycles))],
        phase_seconds={PHASES[i]: ph[i] for i in range(8)} if phase_timing else {},
    )


class _System(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("n", ctypes.c_void_p), ("R", ctypes.c_void_p), ("A", ctypes.c_void_p),
                ("rb", ctypes.c_void_p), ("b", ctypes.c_void_p), ("s", ctypes.c_int32), ("S", ctypes.c_void_p),
                ("rho", ctypes.c_void_p), ("Y", ctypes.c_void_p), ("rx", ctypes.c_void_p), ("X", ctypes.c_void_p),
                ("opts", ctypes.c_void_p), ("x", ctypes.c_void_p), ("x_r", ctypes.c_void_p), ("info", ctypes.c_void_p),
                ("status", ctypes.c_int32), ("ext", ctypes.c_void_p)]


@dataclass
class BatchSystem:
    """One system of a batched solve (cores are CUDA float64 tensors)."""
    A: List[torch.Tensor]
    b: List[torch.Tensor]
    S: List[torch.Tensor]
    X: List[torch.Tensor]
    Y: List[torch.Tensor]
    rx: List[int]
    rho: List[int]
    maxit: int
    tol: float
    q: int = 1
    round_tol: float = 1e-7
    maxrank: int = 0
    restart: int = 0
    final_tol: float = 0.0
    stop_safety: float = 0.1
    rcond: float = 1e-12
    precision: int = PREC_F64
    max_cycles: int = 50
    precond: Optional["Preconditioner"] = None


class GmresOpts(ctypes.Structure):
    _fields_ = [("maxit", ctypes.c_int32), ("maxrank", ctypes.c_int32), ("tol", ctypes.c_double),
                ("final_tol", ctypes.c_double), ("max_round", ctypes.c_double)]


def tt_gmres(A, b, *, maxit: int, tol: float, final_tol: float = 0.0, max_round: float = 0.1, maxrank: int = 0,
             raise_on_error: bool = True) -> SolveResult:
    """TT-GMRES (Alg. 2, ttsg_tt_gmres) with x_0 = 0.  `sketched_history` holds
    the Arnoldi residuals ||r_k|| / ||b|| of every step."""
    d = len(b)
    n = sizes_of(b)
    dev = b[0].device
    opts = GmresOpts(maxit=maxit, maxrank=maxrank, tol=tol, final_tol=final_tol, max_round=max_round)
    nb = ctypes.c_size_t(0)
    _check(lib().ttsg_tt_gmres_workspace_size(d, _i32(n), _i32(op_ranks(A)), _i32(ranks_of(b)), ctypes.byref(opts),
                                              ctypes.byref(nb)), "ttsg_tt_gmres_workspace_size")
    ws = _workspace(nb.value, dev)
    caps = [1] * (d + 1)
    left = 1
    for k in range(1, d):
        left *= n[k - 1]
        right = 1
        for j in range(k, d):
            right *= n[j]
        caps[k] = min(left, right) if maxrank <= 0 else min(left, right, maxrank)
    x = [torch.zeros((caps[k], n[k], caps[k + 1]), dtype=torch.float64, device=dev) for k in range(d)]
    xr = (ctypes.c_int32 * (d + 1))()
    sh = (ctypes.c_double * maxit)()
    rh = (ctypes.c_int32 * maxit)()
    info = SgmresInfo(sketched_history=sh, rank_history=rh)
    rc = lib().ttsg_tt_gmres(d, _i32(n), _i32(op_ranks(A)), _ptrs(A), _i32(ranks_of(b)), _ptrs(b), ctypes.byref(opts),
                             _ptrs(x), xr, ctypes.byref(info), ctypes.c_void_p(ws.data_ptr()), nb, _stream())
    if raise_on_error:
        _check(rc, "ttsg_tt_gmres")
    elif rc < 0:
        return SolveResult(x=[], status=rc, iterations=0, cycles=0, true_residual=float("nan"),
                           sketched_residual=float("nan"), max_rank=0)
    it = info.iterations
    return SolveResult(x=_trim(x, list(xr)), status=rc, iterations=it, cycles=1, true_residual=info.true_residual,
                       sketched_residual=info.sketched_residual, max_rank=info.max_rank,
                       sketched_history=[sh[i] for i in range(min(it, maxit))],
                       rank_history=[rh[i] for i in range(min(it, maxit))])


def sgmres_solve_batched(systems: Sequence[BatchSystem], concurrency: int = 8) -> List[SolveResult]:
    """Solve independent systems concurrently (ttsg_sgmres_solve_batched)."""
    keep = []
    arr = (_System * len(systems))()
    outs = []

    def addr(obj):
        keep.append(obj)
        return ctypes.cast(obj, ctypes.c_void_p)

    for i, q in enumerate(systems):
        d = len(q.b)
        n = sizes_of(q.b)
        dev = q.b[0].device
        opts = SgmresOpts(maxit=q.maxit, restart=q.restart, q=q.q, maxrank=q.maxrank, precision=q.precision,
                          max_cycles=q.max_cycles, tol=q.tol, round_tol=q.round_tol, final_tol=q.final_tol,
                          stop_safety=q.stop_safety, rcond=q.rcond)
        sh = (ctypes.c_double * q.maxit)()
        rh = (ctypes.c_int32 * q.maxit)()
        th = (ctypes.c_double * q.max_cycles)()
        info = SgmresInfo(sketched_history=sh, rank_history=rh, true_history=th, phase_seconds=None)
        x = [torch.zeros((q.rx[k], n[k], q.rx[k + 1]), dtype=torch.float64, device=dev) for k in range(d)]
        xr = (ctypes.c_int32 * (d + 1))()
        keep.extend([opts, info, sh, rh, th, x, xr])
        e = arr[i]
        e.d = d
        e.n = addr(_i32(n))
        e.R = addr(_i32(op_ranks(q.A)))
        e.A = addr(_ptrs(q.A))
        e.rb = addr(_i32(ranks_of(q.b)))
        e.b = addr(_ptrs(q.b))
        e.s = int(q.S[0].shape[0])
        e.S = addr(_ptrs(q.S))
        e.rho = addr(_i32(q.rho))
        e.Y = addr(_ptrs(q.Y))
        e.rx = addr(_i32(q.rx))
        e.X = addr(_ptrs(q.X))
        e.opts = ctypes.cast(ctypes.pointer(opts), ctypes.c_void_p)
        e.x = addr(_ptrs(x))
        e.x_r = ctypes.cast(xr, ctypes.c_void_p)
        e.info = ctypes.cast(ctypes.pointer(info), ctypes.c_void_p)
        if q.precond is not None:
            ext = SgmresExt(ls_mode=LS_PINV, variant=VARIANT_ENHANCED)
            aa, ba, ma = _dbl(q.precond.alpha), _dbl(q.precond.beta), _ptrs(q.precond.M)
            ext.zeta = len(q.precond.alpha)
            ext.alpha = ctypes.cast(aa, ctypes.c_void_p)
            ext.beta = ctypes.cast(ba, ctypes.c_void_p)
            ext.M = ctypes.cast(ma, ctypes.c_void_p)
            keep.extend([ext, aa, ba, ma])
            e.ext = ctypes.cast(ctypes.pointer(ext), ctypes.c_void_p)
        outs.append((x, xr, info, sh, rh, th, q))
    _check(lib().ttsg_sgmres_solve_batched(len(systems), arr, int(concurrency), _stream()),
           "ttsg_sgmres_solve_batched")
    res = []
    for i, (x, xr, info, sh, rh, th, q) in enumerate(outs):
        it = info.iterations
        res.append(SolveResult(
            x=_trim(x, list(xr)), status=arr[i].status, iterations=it, cycles=info.cycles,
            true_residual=info.true_residual, sketched_residual=info.sketched_residual, max_rank=info.max_rank,
            true_residual_is_bound=bool(info.true_residual_is_bound),
            sketched_history=[sh[j] for j in range(min(it, q.maxit))],
            rank_history=[rh[j] for j in range(min(it, q.maxit))],
            true_history=[th[j] for j in range(min(info.cycles, q.max_cycles))]))
    return res

