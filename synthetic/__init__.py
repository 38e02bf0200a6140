"""Seeded synthetic inputs shared by the FP64 oracle and the GPU path.

This module holds no arithmetic of the solver: it only draws random numbers
and writes down the problem data (1-D difference matrices, random TT cores,
sketching matrices) that both sides consume.  Everything returned is a plain
float64 numpy array so the two sides start from bit-identical inputs.

Conventions (0-based):
  * modes mu = 0..d-1, bonds b = 0..d; bond 0 and bond d have rank 1;
  * a TT core of mode mu has shape (r[mu], n[mu], r[mu+1]);
  * the 1-D operator matrices act on the mode index: (A x)[i] = sum_j A[i, j] x[j].

Distributions follow the paper:
  * Khatri-Rao sketch factors S_k in R^{s x n_k} with i.i.d. N(0, s^(-1/d))
    entries, the second argument read as the variance (Sec. 3.1);
  * Gaussian TT-DRM cores with i.i.d. N(0, 1/(l_{k-1} n_k l_k)) entries
    (Definition 3.1);
  * right-hand sides with i.i.d. Gaussian cores; core k is scaled by
    1/sqrt(n_k r_k) so that E||b||^2 = 1 (the workloads ask for unit-norm
    right-hand sides; every reported residual is relative, so only the
    direction of b matters).
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

SEED_BASE = 240909471


def rng_for(config_index: int, stream: int = 0) -> np.random.Generator:
    """Generator for one workload; `stream` separates independent draws."""
    return np.random.default_rng([SEED_BASE + config_index, stream])


# ----------------------------------------------------------------------------
# 1-D matrices of the model problems (Sec. 5.1.1 and the workload list)
# ----------------------------------------------------------------------------

def laplacian_1d(n: int) -> np.ndarray:
    """(n+1)^2 * tridiag(-1, 2, -1): minus the second difference, h = 1/(n+1).

    The paper writes the diffusion block as K/h^2 tridiag(1,-2,1) for the
    equation K Lap u + ... + f = 0; moving it to the SPD form A x = b flips
    the sign, which is what is used here (K = 1)."""
    h2 = float(n + 1) ** 2
    A = np.zeros((n, n))
    idx = np.arange(n)
    A[idx, idx] = 2.0 * h2
    A[idx[:-1], idx[:-1] + 1] = -h2
    A[idx[1:], idx[1:] - 1] = -h2
    return A


def upwind_1d(n: int, w: float) -> np.ndarray:
    """w/h * (I - superdiagonal), h = 1/(n+1): the first-difference block of
    Sec. 5.1.1 with its sign flipped to match the SPD diffusion block."""
    A = np.zeros((n, n))
    idx = np.arange(n)
    A[idx, idx] = w * (n + 1)
    A[idx[:-1], idx[:-1] + 1] = -w * (n + 1)
    return A


def potential_1d(n: int) -> np.ndarray:
    """diag(sin(pi x_i)), x_i = i/(n+1), i = 1..n."""
    x = np.arange(1, n + 1) / (n + 1.0)
    return np.diag(np.sin(np.pi * x))


def convdiff_1d(n: int, K: float = 1e-2, w: float = 1e-2, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """Mode matrix of the convection-diffusion problem of Sec. 5.1.1 on [lo, hi]
    with h = (hi - lo)/(n+1), written for the SPD-signed system A x = f:
    K/h^2 tridiag(-1, 2, -1) + w/h (I - superdiagonal), i.e. minus the paper's
    L + D_i (its equation reads (sum_i (L + D_i)) x + f = 0)."""
    h = (hi - lo) / (n + 1.0)
    A = np.zeros((n, n))
    idx = np.arange(n)
    A[idx, idx] = 2.0 * K / h ** 2 + w / h
    A[idx[:-1], idx[:-1] + 1] = -K / h ** 2 - w / h
    A[idx[1:], idx[1:] - 1] = -K / h ** 2
    return A


def gauss_source_1d(n: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """exp(-10 x_i^2) at the interior grid points x_i = lo + i h, i = 1..n: one
    factor of the rank-1 source f(x) = exp(-10 ||x||^2) of Sec. 5.1.1."""
    h = (hi - lo) / (n + 1.0)
    x = lo + h * np.arange(1, n + 1)
    return np.exp(-10.0 * x ** 2)


def markov_rates(rng: np.random.Generator, d: int, n: int):
    """Forward and backward rates of the d random walks of Sec. 5.1.2, each drawn
    independently from U[1, 2]: eta[k][i] from state i to i+1, mu[k][i] from
    state i to i-1 (0-based states 0..n-1)."""
    eta = [rng.uniform(1.0, 2.0, size=n) for _ in range(d)]
    mu = [rng.uniform(1.0, 2.0, size=n) for _ in range(d)]
    return eta, mu


def markov_walk_1d(eta: np.ndarray, mu: np.ndarray) -> np.ndarray:
    """Generator block Q_i of one random walk, row = source state, column =
    target state: Q[i, i+1] = eta[i], Q[i, i-1] = mu[i], Q[i, i] = -(eta[i] +
    mu[i]).  The walk's boundary moves (eta of the last state, mu of the first)
    leave the chain, so -Q_i is a nonsingular M-matrix."""
    n = len(eta)
    Q = np.zeros((n, n))
    idx = np.arange(n)
    Q[idx, idx] = -(eta + mu)
    Q[idx[:-1], idx[:-1] + 1] = eta[:-1]
    Q[idx[1:], idx[1:] - 1] = mu[1:]
    return Q


def markov_sync_1d(n: int):
    """The two one-entry factors of a synchronized joint failure of Sec. 5.1.2:
    J moves a system from state n-2 to state n-1 (0-based), P = e_{n-2} e_{n-2}^T
    is the matching diagonal entry of the row-sum correction D."""
    J = np.zeros((n, n))
    J[n - 2, n - 1] = 1.0
    P = np.zeros((n, n))
    P[n - 2, n - 2] = 1.0
    return J, P


# ----------------------------------------------------------------------------
# Random TT data
# ----------------------------------------------------------------------------

def gaussian_tt(rng: np.random.Generator, ns: List[int], ranks: List[int]) -> List[np.ndarray]:
    """Random TT with i.i.d. Gaussian cores; ranks has length d+1 with ranks[0]=ranks[d]=1.
    Core k is scaled by 1/sqrt(n_k r_{k+1}) so that E||x||^2 = 1."""
    d = len(ns)
    assert len(ranks) == d + 1 and ranks[0] == 1 and ranks[d] == 1
    cores = []
    for k in range(d):
        shape = (ranks[k], ns[k], ranks[k + 1])
        cores.append(rng.standard_normal(shape) / np.sqrt(ns[k] * ranks[k + 1]))
    return cores


def tt_drm(rng: np.random.Generator, ns: List[int], ranks: List[int], first: int, last: int) -> List[np.ndarray]:
    """Gaussian TT-DRM cores for modes first..last-1 (Definition 3.1).

    `ranks` is indexed by bond (length d+1); core k has shape
    (ranks[k], n_k, ranks[k+1]) and variance 1/(ranks[k] n_k ranks[k+1])."""
    cores = []
    for k in range(first, last):
        shape = (ranks[k], ns[k], ranks[k + 1])
        var = 1.0 / (ranks[k] * ns[k] * ranks[k + 1])
        cores.append(rng.standard_normal(shape) * np.sqrt(var))
    return cores


def kr_factors(rng: np.random.Generator, s: int, ns: List[int]) -> List[np.ndarray]:
    """Khatri-Rao sketch factors S_k (s x n_k), entries N(0, s^(-1/d)) (variance)."""
    d = len(ns)
    std = np.sqrt(float(s) ** (-1.0 / d))
    return [rng.standard_normal((s, n)) * std for n in ns]


def bond_caps(ns: List[int], cap: int) -> List[int]:
    """min(cap, prod_{k<b} n_k, prod_{k>=b} n_k) for every bond b = 0..d."""
    d = len(ns)
    out = []
    for b in range(d + 1):
        left = int(np.prod(ns[:b], dtype=np.float64)) if b > 0 else 1
        right = int(np.prod(ns[b:], dtype=np.float64)) if b < d else 1
        out.append(int(min(cap, left, right)))
    return out


def stta_ranks(ns: List[int], cap: int, oversample: int, rho_max: Optional[int] = None):
    """Target ranks r_X (right DRM X) and left sketch ranks rho (left DRM Y).

    r_X,b = min(cap, prod_{k<b} n_k, prod_{k>=b} n_k); rho_b = r_X,b + oversample,
    clipped to prod_{k<b} n_k (the number of rows of Y_{<=b}) and to rho_max."""
    rx = bond_caps(ns, cap)
    d = len(ns)
    rho = []
    for b in range(d + 1):
        if b == 0 or b == d:
            rho.append(1)
            continue
        left = float(np.prod(ns[:b], dtype=np.float64))
        v = rx[b] + oversample
        if rho_max is not None:
            v = min(v, rho_max)
        v = int(min(v, left))
        rho.append(max(v, rx[b]))
    return rx, rho


# ----------------------------------------------------------------------------
# Workloads
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Workload:
    """One linear system A x = b in TT form plus the random sketches of the method.

    terms: list of (kind, per-mode 1-D matrices) making up a Kronecker sum
      sum_k I x ... x M_k x ... x I for each term; `op_rank` is the TT rank
      with which that sum is to be represented (2 for one term, 3 for two).
    """
    name: str
    d: int
    ns: List[int]
    terms: List[List[np.ndarray]]
    op_rank: int
    b: List[np.ndarray]
    S: List[np.ndarray]
    X: List[np.ndarray]          # DRM cores for modes 1..d-1 (right sketch)
    Y: List[np.ndarray]          # DRM cores for modes 0..d-2 (left sketch)
    rx: List[int]
    rho: List[int]
    cap: int
    s: int
    q: int
    maxit: int
    restart: int
    tol: float
    round_tol: float
    stop_safety: float
    extra: dict = dataclasses.field(default_factory=dict)


def _sketches(rng, ns, s, cap, oversample, rho_max=None):
    S = kr_factors(rng, s, ns)
    rx, rho = stta_ranks(ns, cap, oversample, rho_max)
    d = len(ns)
    X = tt_drm(rng, ns, rx, 1, d)
    Y = tt_drm(rng, ns, rho, 0, d - 1)
    return S, X, Y, rx, rho


def laplace_plain(d: int, n: int, *, config_index: int = 0, b_rank: int = 1, b_ones: bool = False,
                  cap: int = 64, s: int = 40, q: int = 2, maxit: int = 200, restart: int = 0,
                  tol: float = 1e-6, round_tol: float = 1e-8, stop_safety: float = 0.1,
                  oversample: int = 20, stream: int = 0, name: str = "laplace") -> Workload:
    """Pure d-dimensional Laplacian (rank-2 TT operator) with a random or all-ones rhs."""
    rng = rng_for(config_index, stream)
    ns = [n] * d
    L = laplacian_1d(n)
    if b_ones:
        b = [np.ones((1, n, 1)) for _ in range(d)]
    else:
        b = gaussian_tt(rng, ns, [1] + [b_rank] * (d - 1) + [1])
    S, X, Y, rx, rho = _sketches(rng, ns, s, cap, oversample)
    return Workload(name, d, ns, [[L] * d], 2, b, S, X, Y, rx, rho, cap, s, q, maxit, restart,
                    tol, round_tol, stop_safety)


def config_c1() -> Workload:
    """FP64: d=5, n=16, Laplacian, b = all-ones rank 1, restart 20, s = 40, q = 2,
    rounding tol 1e-8, stop at relative residual 1e-6.  The workload sets no rank
    cap, so the STTA target ranks are the full ranks min(16^b, 16^(5-b))."""
    return laplace_plain(5, 16, config_index=0, b_ones=True, cap=256, s=40, q=2, maxit=400,
                         restart=20, tol=1e-6, round_tol=1e-8, name="laplace_d5_n16")


def config_c2(d: int = 10, n: int = 64, s: int = 1000, maxit: int = 500) -> Workload:
    """d=10, n=64: Laplacian + 0.1 x upwind convection in mode 1 (rank-3 TT),
    b Gaussian rank 4, ranks capped at 64, s = 1000, q = 1; the sketched residual
    is compared with 0.3 tol (the factor the paper uses for its n = 64 runs)."""
    rng = rng_for(1)
    ns = [n] * d
    L = laplacian_1d(n)
    conv = [upwind_1d(n, 0.1)] + [np.zeros((n, n))] * (d - 1)
    b = gaussian_tt(rng, ns, [1] + [4] * (d - 1) + [1])
    S, X, Y, rx, rho = _sketches(rng, ns, s, 64, 20)
    return Workload(f"convdiff_d{d}_n{n}", d, ns, [[L] * d, conv], 3, b, S, X, Y, rx, rho, 64, s, 1,
                    maxit, 0, 1e-6, 1e-7, 0.3)


def config_c3_systems(count: int = 64):
    """Batched: `count` systems, d ~ U{6..12}, n ~ U{32,64,128}, b rank ~ U{2..8}, caps 32."""
    rng = rng_for(2)
    out = []
    for i in range(count):
        d = int(rng.integers(6, 13))
        n = int(rng.choice([32, 64, 128]))
        rb = int(rng.integers(2, 9))
        out.append((d, n, rb))
    return out


def config_c3_system(i: int, d: int, n: int, rb: int, s: int = 1000, maxit: int = 500, cap: int = 32) -> Workload:
    rng = rng_for(2, 1 + i)
    ns = [n] * d
    L = laplacian_1d(n)
    b = gaussian_tt(rng, ns, [1] + [rb] * (d - 1) + [1])
    S, X, Y, rx, rho = _sketches(rng, ns, s, cap, 20)
    return Workload(f"batch{i}_d{d}_n{n}", d, ns, [[L] * d], 2, b, S, X, Y, rx, rho, cap, s, 1,
                    maxit, 0, 1e-6, 1e-7, 0.1)


def config_c4(d: int = 8, n: int = 64):
    """Differentiation workload: theta_k ~ U[0.5, 2], b rank 3, x_target rank 2."""
    rng = rng_for(3)
    theta = rng.uniform(0.5, 2.0, size=d)
    ns = [n] * d
    b = gaussian_tt(rng, ns, [1] + [3] * (d - 1) + [1])
    xt = gaussian_tt(rng, ns, [1] + [2] * (d - 1) + [1])
    S, X, Y, rx, rho = _sketches(rng, ns, 1000, 64, 20)
    return dict(theta=theta, ns=ns, d=d, n=n, L=laplacian_1d(n), b=b, x_target=xt, S=S, X=X, Y=Y,
                rx=rx, rho=rho)


def config_c5(d: int = 20, n: int = 128, s: int = 2000, maxit: int = 60, restart: int = 20) -> Workload:
    """Large: d=20, n=128, Laplacian + sum_k diag(sin(pi x_k)) (rank-3 TT),
    b Gaussian rank 8, ranks capped at 128, left sketch ranks <= 160.

    Solved with the exponential-sum right preconditioner of the operator's own
    Kronecker sum (mode matrices L + V, extra["mode_matrices"]) at relative
    accuracy extra["precond_tol"] = 0.02 on the sum's spectrum interval (13
    terms; 4 iterations, against 6 with 8 terms at 0.1); restart
    cycles of 20 keep the stored FP64 sketches of the basis (about 420 MB per
    vector at these ranks) bounded."""
    rng = rng_for(4)
    ns = [n] * d
    L = laplacian_1d(n)
    V = potential_1d(n)
    b = gaussian_tt(rng, ns, [1] + [8] * (d - 1) + [1])
    S = kr_factors(rng, s, ns)
    rx, rho = stta_ranks(ns, 128, 20, rho_max=160)
    X = tt_drm(rng, ns, rx, 1, d)
    Y = tt_drm(rng, ns, rho, 0, d - 1)
    return Workload(f"potential_d{d}_n{n}", d, ns, [[L] * d, [V] * d], 3, b, S, X, Y, rx, rho, 128,
                    s, 1, maxit, restart, 1e-6, 1e-7, 0.1,
                    extra={"mode_matrices": [L + V] * d, "precond_tol": 0.02})


def markov_chain(d: int, n: int, *, config_index: int = 5, rate: float = 0.1, s: int = 200,
                 cap: int = 64, oversample: int = 20, stream: int = 0) -> dict:
    """Synchronized Markov chain of Sec. 5.1.2: d random walks with n states and
    U[1, 2] rates, neighbouring systems failing together at `rate`; right-hand
    side e (all ones, rank 1).  Returns the problem data (per-mode generator
    blocks Q_k, the one-entry factors J and P) and the sketches of the method."""
    rng = rng_for(config_index, stream)
    ns = [n] * d
    eta, mu = markov_rates(rng, d, n)
    Q = [markov_walk_1d(e, m) for e, m in zip(eta, mu)]
    J, P = markov_sync_1d(n)
    b = [np.ones((1, n, 1)) for _ in range(d)]
    S, X, Y, rx, rho = _sketches(rng, ns, s, cap, oversample)
    return dict(d=d, n=n, ns=ns, Q=Q, J=J, P=P, rate=rate, b=b, S=S, X=X, Y=Y, rx=rx, rho=rho, s=s,
                cap=cap)
